// Serving loop: continuous batching of all-bins scans over a resident index.
//
// Requests (read sets in host memory) are copied into a pinned host arena at
// submit and queued. A scheduler thread
//   1. admits queued requests in arrival order while fewer than max_inflight
//      are admitted and the request's device footprint (inputs, tokens,
//      thresholds, descriptors and its pass masks) fits the free bytes of the
//      device arena, a block of HBM sized from free device memory at creation;
//   2. prepares each admitted request on a prep stream: H2D copies, status
//      reset, tokenisation + thresholds, and one descriptor per read
//      (token list, mask row, token count, threshold);
//   3. forms launches: the continuous policy takes up to max_batch_reads reads
//      from all prepared requests, at most slice_reads from each, gathers
//      their descriptors into a launch buffer, orders them by length (so a
//      wavefront's reads have equal loop counts: reads of 100, 150 and 250 bp
//      arrive mixed) and runs the all-bins scan on one of n_streams streams,
//      so requests that arrive while others run share launches and overlap on
//      the device; the plain policy runs each request alone, in arrival
//      order, as one launch on one stream;
//   4. completes a request when the launches holding its last reads have
//      finished, recording its latency from submit.
// Results stay in device memory until the client releases them. The
// arithmetic is the scan kernel's: a served request's masks are bit-identical
// to grim_filter_scan on the same reads.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "grim_internal.h"
#include "serve_core.h"

namespace grim {

int status_to_error(uint32_t st);

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

constexpr int kMaxSegs = 64;

struct SegTable {
  uint32_t n_seg;
  uint32_t total;
  struct {
    const ReadDesc* src;
    uint32_t first;
    uint32_t dst;
  } seg[kMaxSegs];
  uint32_t end[kMaxSegs];  // exclusive end (in launch positions) of each segment
};

// descriptor of read r of one request
__global__ void k_make_desc(const int64_t* offsets, const uint32_t* tokens, const int32_t* thr, uint32_t* mask,
                            uint64_t W, uint32_t q, uint64_t n, ReadDesc* desc) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t o0 = offsets[r], o1 = offsets[r + 1];
  ReadDesc d;
  d.tok = tokens + token_base(o0, r);
  d.out = mask + r * W;
  d.ntok = (uint32_t)(o1 - o0 - q + 1);
  d.T = thr[r];
  desc[r] = d;
}

// gather the descriptors of a launch's segments into one array
__global__ void k_gather_desc(SegTable t, ReadDesc* dst) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= t.total) return;
  uint32_t s = 0;
  while (s + 1 < t.n_seg && k >= t.end[s]) ++s;
  const uint32_t j = k - t.seg[s].dst;
  dst[k] = t.seg[s].src[t.seg[s].first + j];
}

// Order a launch's reads by their number of 32-token blocks, longest first,
// so the reads sharing a wavefront have (nearly) the same loop count and the
// long ones start first. One workgroup; counting sort over 64 buckets.
__global__ __launch_bounds__(1024) void k_sort_desc(const ReadDesc* desc, uint32_t n, uint32_t* order) {
  __shared__ uint32_t hist[64];
  if (threadIdx.x < 64) hist[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
    const uint32_t b = min((desc[k].ntok + 31) >> 5, 63u);
    atomicAdd(&hist[63 - b], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < 64; ++i) {
      const uint32_t c = hist[i];
      hist[i] = acc;
      acc += c;
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
    const uint32_t b = min((desc[k].ntok + 31) >> 5, 63u);
    order[atomicAdd(&hist[63 - b], 1u)] = k;
  }
}

enum class RState { Queued, Prepping, Active, Done, Failed, Canceled };

struct Request {
  uint64_t ticket = 0;
  RState state = RState::Queued;
  uint64_t n_reads = 0, n_bases = 0;
  uint32_t edits_kind = 0;  // 0 none, 1 max_edits, 2 err_permille
  uint32_t err_all = 0;
  uint64_t host_off = 0;
  bool host_held = false;
  uint64_t dev_off = 0;
  bool dev_held = false;
  serve::Footprint fp{};
  hipEvent_t ready = nullptr;
  uint32_t* status_host = nullptr;  // pinned word the prep stream copies the status into
  uint64_t done_reads = 0;
  uint32_t launches_in_flight = 0;
  bool cancel_requested = false;
  bool admitted_once = false;
  int status = GRIM_OK;
  Clock::time_point t_submit, t_admit, t_done;
  bool released = false;
};

struct LaunchSlot {
  ReadDesc* desc = nullptr;
  uint32_t* order = nullptr;  // launch position -> descriptor, sorted by length
  hipEvent_t done = nullptr;
  bool busy = false;
  uint32_t stream = 0;
  std::vector<serve::Segment> segs;
};

}  // namespace
}  // namespace grim

struct grim_server {
  const grim_index* idx = nullptr;
  grim_serve_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work;   // wakes the scheduler
  std::condition_variable cv_done;   // wakes waiters
  std::thread thread;
  bool stop = false;
  // memory
  uint8_t* dev_base = nullptr;
  grim::serve::Arena dev_arena;
  uint8_t* host_base = nullptr;
  grim::serve::Arena host_arena;
  uint32_t* status_pinned = nullptr;  // one word per in-flight prep
  std::vector<uint32_t> status_free;
  // streams and launches
  hipStream_t prep = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<grim::LaunchSlot> slots;
  uint32_t next_stream = 0;
  // requests
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, std::unique_ptr<grim::Request>> reqs;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> prepping;
  grim::serve::BatchFormer former;
  uint32_t admitted = 0;  // prepping + active
  // stats
  uint64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_rejected = 0, n_canceled = 0, reads_completed = 0;
  uint64_t launches = 0, peak_dev = 0, shared_launches = 0, max_reqs_per_launch = 0;
  std::vector<double> latencies;
  bool have_first = false;
  grim::Clock::time_point t_first_submit, t_last_done;
  int device = 0;
  std::string fatal;  // a HIP failure that stopped the scheduler
  // test hook, read at creation from GRIM_SERVE_TEST_FAIL_LAUNCH: launch
  // number n >= 1 and every later one report a launch failure from the host
  // without launching anything (0: off), so the failure path can be tested
  // without a device fault
  uint64_t fail_launch_at = 0;
};

namespace grim {
namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void finish(grim_server* S, Request& r, RState st, int code) {
  r.state = st;
  r.status = code;
  r.t_done = Clock::now();
  if (r.host_held) {
    S->host_arena.release(r.host_off);
    r.host_held = false;
  }
  if (st == RState::Done) {
    S->n_completed++;
    S->reads_completed += r.n_reads;
    S->latencies.push_back(ms_since(r.t_submit, r.t_done));
    S->t_last_done = r.t_done;
  } else {
    // failed or cancelled requests give their device block back at once
    if (r.dev_held) {
      S->dev_arena.release(r.dev_off);
      r.dev_held = false;
    }
    if (st == RState::Failed) S->n_failed++;
    else S->n_canceled++;
  }
  if (r.ready) {
    (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
  }
  if (r.status_host) {
    S->status_free.push_back((uint32_t)(r.status_host - S->status_pinned));
    r.status_host = nullptr;
  }
  S->cv_done.notify_all();
}

// Start preparing an admitted request on the prep stream. Caller holds mu.
hipError_t start_prep(grim_server* S, Request& r) {
  const grim_index* idx = S->idx;
  uint8_t* blk = S->dev_base + r.dev_off;
  const uint8_t* hblk = S->host_base + r.host_off;
  const serve::Footprint& f = r.fp;
  hipStream_t s = S->prep;
  hipError_t e;
  // host block layout mirrors the device block up to the edits
  if ((e = hipMemcpyAsync(blk + f.off_bases, hblk + f.off_bases, r.n_bases, hipMemcpyHostToDevice, s))) return e;
  if ((e = hipMemcpyAsync(blk + f.off_offsets, hblk + f.off_offsets, (r.n_reads + 1) * 8, hipMemcpyHostToDevice, s)))
    return e;
  if (r.edits_kind &&
      (e = hipMemcpyAsync(blk + f.off_edits, hblk + f.off_edits, r.n_reads * 2, hipMemcpyHostToDevice, s)))
    return e;
  uint32_t* status = reinterpret_cast<uint32_t*>(blk + f.off_status);
  if ((e = launch_zero_words(status, 8, s))) return e;
  TokArgs t{};
  t.bases = blk + f.off_bases;
  t.offsets = reinterpret_cast<const int64_t*>(blk + f.off_offsets);
  t.n_reads = r.n_reads;
  t.n_bases = r.n_bases;
  t.max_edits = r.edits_kind == 1 ? reinterpret_cast<const uint16_t*>(blk + f.off_edits) : nullptr;
  t.err_pm = r.edits_kind == 2 ? reinterpret_cast<const uint16_t*>(blk + f.off_edits) : nullptr;
  t.err_pm_all = r.err_all;
  t.q = idx->q;
  t.overlap = idx->O;
  t.flags = S->cfg.flags;
  t.max_tokens = 65535u;
  t.tok_shift = scan_token_shift(idx->q);
  t.tokens = reinterpret_cast<uint32_t*>(blk + f.off_tokens);
  t.thr = reinterpret_cast<int32_t*>(blk + f.off_thr);
  t.status = status;
  if ((e = launch_tokenize(t, s))) return e;
  hipLaunchKernelGGL(k_make_desc, dim3((unsigned)((r.n_reads + 255) / 256)), dim3(256), 0, s, t.offsets, t.tokens,
                     t.thr, reinterpret_cast<uint32_t*>(blk + f.off_mask), idx->W, idx->q, r.n_reads,
                     reinterpret_cast<ReadDesc*>(blk + f.off_desc));
  if ((e = hipGetLastError())) return e;
  if ((e = hipMemcpyAsync(r.status_host, status, 4, hipMemcpyDeviceToHost, s))) return e;
  if ((e = hipEventCreateWithFlags(&r.ready, hipEventDisableTiming))) return e;
  return hipEventRecord(r.ready, s);
}

// Launch one batch of segments on a free slot. Caller holds mu.
hipError_t start_launch(grim_server* S, LaunchSlot& L, std::vector<serve::Segment>&& segs) {
  const grim_index* idx = S->idx;
  if (S->fail_launch_at && S->launches + 1 >= S->fail_launch_at) return hipErrorLaunchFailure;
  SegTable t{};
  uint32_t total = 0;
  for (auto& sg : segs) {
    Request& r = *S->reqs[sg.req];
    auto& e = t.seg[t.n_seg];
    e.src = reinterpret_cast<const ReadDesc*>(S->dev_base + r.dev_off + r.fp.off_desc);
    e.first = (uint32_t)sg.first;
    e.dst = total;
    total += (uint32_t)sg.count;
    t.end[t.n_seg] = total;
    t.n_seg++;
  }
  t.total = total;
  L.stream = S->cfg.policy == GRIM_SERVE_PLAIN ? 0 : (S->next_stream++ % (uint32_t)S->streams.size());
  hipStream_t s = S->streams[L.stream];
  hipLaunchKernelGGL(k_gather_desc, dim3((total + 255) / 256), dim3(256), 0, s, t, L.desc);
  hipError_t e = hipGetLastError();
  if (e) return e;
  const bool sorted = S->cfg.policy == GRIM_SERVE_CONTINUOUS;
  if (sorted) {
    hipLaunchKernelGGL(k_sort_desc, dim3(1), dim3(1024), 0, s, L.desc, total, L.order);
    if ((e = hipGetLastError())) return e;
  }
  ScanArgs a{};
  a.desc = L.desc;
  a.read_order = sorted ? L.order : nullptr;
  a.tm = idx->tm;
  a.row_words = idx->row_words;
  a.R4 = idx->R4;
  a.q = idx->q;
  a.nb = idx->nb;
  a.W = idx->W;
  a.n_reads = total;
  a.status = nullptr;
  if ((e = launch_scan_allbins(a, idx->scan_cfg, s))) return e;
  if ((e = hipEventRecord(L.done, s))) return e;
  for (auto& sg : segs) S->reqs[sg.req]->launches_in_flight++;
  S->shared_launches += segs.size() > 1;
  S->max_reqs_per_launch = std::max<uint64_t>(S->max_reqs_per_launch, segs.size());
  L.segs = std::move(segs);
  L.busy = true;
  S->launches++;
  return hipSuccess;
}

void scheduler(grim_server* S) {
  DeviceGuard dg(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progress = false;
    // 0. after a device failure nothing more is admitted: queued requests fail
    if (!S->fatal.empty()) {
      while (!S->queue.empty()) {
        auto qit = S->reqs.find(S->queue.front());
        S->queue.pop_front();
        if (qit != S->reqs.end() && qit->second->state == RState::Queued)
          finish(S, *qit->second, RState::Failed, GRIM_EDEVICE);
        progress = true;
      }
    }
    // 1. admission, in arrival order
    while (S->fatal.empty() && !S->queue.empty() && S->admitted < S->cfg.max_inflight && !S->status_free.empty()) {
      auto qit = S->reqs.find(S->queue.front());
      if (qit == S->reqs.end() || qit->second->state != RState::Queued) {  // cancelled (and released) while queued
        S->queue.pop_front();
        continue;
      }
      Request& r = *qit->second;
      uint64_t off = 0;
      if (!S->dev_arena.alloc(r.fp.total, &off)) {
        if (S->dev_arena.used() == 0) {  // would not fit even alone
          S->queue.pop_front();
          S->n_rejected++;
          finish(S, r, RState::Failed, GRIM_ENOMEM);
          progress = true;
          continue;
        }
        break;  // head of line waits for memory
      }
      S->queue.pop_front();
      r.dev_off = off;
      r.dev_held = true;
      S->peak_dev = std::max(S->peak_dev, S->dev_arena.used());
      r.status_host = S->status_pinned + S->status_free.back();
      S->status_free.pop_back();
      r.t_admit = Clock::now();
      r.admitted_once = true;
      r.state = RState::Prepping;
      S->admitted++;
      hipError_t e = start_prep(S, r);
      if (e != hipSuccess) {
        S->fatal = hipGetErrorString(e);
        S->admitted--;
        finish(S, r, RState::Failed, GRIM_EDEVICE);
      } else {
        S->prepping.push_back(r.ticket);
      }
      progress = true;
    }
    // 2. prepared requests join the batch former (or fail on bad reads)
    for (size_t i = 0; i < S->prepping.size();) {
      Request& r = *S->reqs[S->prepping[i]];
      const hipError_t q = hipEventQuery(r.ready);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess && S->fatal.empty()) S->fatal = hipGetErrorString(q);
      S->prepping.erase(S->prepping.begin() + (long)i);
      progress = true;
      if (r.host_held) {
        S->host_arena.release(r.host_off);
        r.host_held = false;
      }
      const uint32_t st = q == hipSuccess ? *r.status_host : 0u;
      if (r.cancel_requested) {
        S->admitted--;
        finish(S, r, RState::Canceled, GRIM_ECANCELED);
      } else if (!S->fatal.empty()) {
        // the server stopped while this request was prepared
        S->admitted--;
        finish(S, r, RState::Failed, GRIM_EDEVICE);
      } else if (st != 0) {
        S->admitted--;
        finish(S, r, RState::Failed, status_to_error(st));
      } else {
        r.state = RState::Active;
        S->former.add(r.ticket, r.n_reads);
      }
    }
    // 3. launches
    for (auto& L : S->slots) {
      if (L.busy || S->former.empty() || !S->fatal.empty()) continue;
      // the plain policy takes one whole request per launch, in arrival order
      const uint64_t maxr = S->cfg.policy == GRIM_SERVE_PLAIN ? S->cfg.max_request_reads : S->cfg.max_batch_reads;
      const uint64_t slice = S->cfg.policy == GRIM_SERVE_PLAIN ? S->cfg.max_request_reads : S->cfg.slice_reads;
      const size_t max_segs = S->cfg.policy == GRIM_SERVE_PLAIN ? 1 : (size_t)kMaxSegs;
      std::vector<serve::Segment> segs = S->former.next_batch(maxr, slice, max_segs);
      if (segs.empty()) continue;
      std::vector<serve::Segment> kept = segs;
      hipError_t e = start_launch(S, L, std::move(segs));
      progress = true;
      if (e != hipSuccess) {
        // the device refused a launch: stop serving, fail what is left
        S->fatal = hipGetErrorString(e);
        for (auto& sg : kept) {
          Request& r = *S->reqs[sg.req];
          r.cancel_requested = true;
          r.status = GRIM_EDEVICE;
        }
        for (auto& kv : S->reqs) {
          Request& r = *kv.second;
          if (r.state != RState::Active) continue;
          r.cancel_requested = true;
          r.status = GRIM_EDEVICE;
          S->former.remove(r.ticket);
          if (r.launches_in_flight == 0) {
            S->admitted--;
            finish(S, r, RState::Failed, GRIM_EDEVICE);
          }
        }
        break;
      }
    }
    // 4. completions
    for (auto& L : S->slots) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) continue;
      L.busy = false;
      progress = true;
      if (q != hipSuccess) {
        // the launch failed on the device: its requests fail and serving stops
        if (S->fatal.empty()) S->fatal = hipGetErrorString(q);
        for (auto& sg : L.segs) S->reqs[sg.req]->status = GRIM_EDEVICE;
      }
      for (auto& sg : L.segs) {
        Request& r = *S->reqs[sg.req];
        r.done_reads += sg.count;
        r.launches_in_flight--;
        if (r.launches_in_flight == 0 && (r.done_reads == r.n_reads || r.cancel_requested)) {
          S->admitted--;
          if (r.status == GRIM_EDEVICE) finish(S, r, RState::Failed, GRIM_EDEVICE);
          else if (r.cancel_requested && r.done_reads != r.n_reads) finish(S, r, RState::Canceled, GRIM_ECANCELED);
          else finish(S, r, RState::Done, GRIM_OK);
        }
      }
      L.segs.clear();
    }
    if (!S->fatal.empty() && !S->former.empty()) {
      // requests waiting for a launch that will not come
      for (auto& kv : S->reqs) {
        Request& r = *kv.second;
        if (r.state != RState::Active) continue;
        r.cancel_requested = true;
        r.status = GRIM_EDEVICE;
        S->former.remove(r.ticket);
        if (r.launches_in_flight == 0) {
          S->admitted--;
          finish(S, r, RState::Failed, GRIM_EDEVICE);
        }
      }
      progress = true;
    }
    const bool busy = std::any_of(S->slots.begin(), S->slots.end(), [](const LaunchSlot& L) { return L.busy; });
    const bool idle = S->queue.empty() && S->prepping.empty() && S->former.empty() && !busy;
    if (S->stop && (idle || (!S->fatal.empty() && S->queue.empty() && S->prepping.empty() && !busy))) break;
    if (!progress) {
      if (idle) S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      else S->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

int fill_result(grim_server* S, const Request& r, grim_result* out) {
  std::memset(out, 0, sizeof *out);
  out->ticket = r.ticket;
  out->status = r.status;
  out->n_reads = r.n_reads;
  out->mask_words = S->idx->W;
  out->mask = (r.state == RState::Done && r.dev_held)
                  ? reinterpret_cast<const uint32_t*>(S->dev_base + r.dev_off + r.fp.off_mask)
                  : nullptr;
  out->latency_ms = ms_since(r.t_submit, r.t_done);
  out->queue_ms = r.admitted_once ? ms_since(r.t_submit, r.t_admit) : 0.0;
  return r.status;
}

void release_all(grim_server* S) {
  if (S->dev_base) (void)hipFree(S->dev_base);
  if (S->host_base) (void)hipHostFree(S->host_base);
  if (S->status_pinned) (void)hipHostFree(S->status_pinned);
  for (auto& L : S->slots) {
    if (L.desc) (void)hipFree(L.desc);
    if (L.order) (void)hipFree(L.order);
    if (L.done) (void)hipEventDestroy(L.done);
  }
  for (auto s : S->streams) (void)hipStreamDestroy(s);
  if (S->prep) (void)hipStreamDestroy(S->prep);
  for (auto& kv : S->reqs)
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
}

}  // namespace
}  // namespace grim

using namespace grim;

extern "C" int grim_serve_create(const grim_index* idx, const grim_serve_config* cfg_in, grim_server** out) {
  clear_error();
  if (!idx || !out) return set_error(GRIM_EINVAL, "NULL argument");
  *out = nullptr;
  if (!(idx->layout & GRIM_LAYOUT_TM)) return set_error(GRIM_EINVAL, "serving needs the token-major layout");
  grim_serve_config c = cfg_in ? *cfg_in : grim_serve_config{};
  if (c.policy > GRIM_SERVE_PLAIN) return set_error(GRIM_EINVAL, "bad policy");
  if (c.flags & ~GRIM_READS_ALLOW_SHORT_OVERLAP) return set_error(GRIM_EINVAL, "unknown flags");
  if (!c.max_inflight) c.max_inflight = 64;
  if (!c.max_batch_reads) c.max_batch_reads = 131072;
  if (!c.slice_reads) c.slice_reads = 32768;
  if (!c.n_streams) c.n_streams = 2;
  if (!c.max_request_reads) c.max_request_reads = 65536;
  if (!c.host_arena_bytes) c.host_arena_bytes = 1ull << 30;
  if (c.max_inflight > 4096 || c.n_streams > 16 || c.max_batch_reads > (1u << 22) || c.max_request_reads > (1u << 22))
    return set_error(GRIM_EINVAL, "configuration out of range");
  if (c.policy == GRIM_SERVE_PLAIN) c.n_streams = 1;
  DeviceGuard dg(idx->device);
  std::unique_ptr<grim_server> S(new grim_server);
  S->idx = idx;
  S->device = idx->device;
  auto fail = [&](int code, const char* what, hipError_t e) {
    release_all(S.get());
    return set_error(code, "%s: %s", what, hipGetErrorString(e));
  };
  if (!c.arena_bytes) {
    size_t fr = 0, tot = 0;
    hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e) return set_error(GRIM_EDEVICE, "hipMemGetInfo: %s", hipGetErrorString(e));
    if (fr <= c.reserve_bytes + (64ull << 20)) return set_error(GRIM_ENOMEM, "no free device memory to serve from");
    c.arena_bytes = (fr - c.reserve_bytes) / 4096 * 4096;
  }
  S->cfg = c;
  if (const char* t = std::getenv("GRIM_SERVE_TEST_FAIL_LAUNCH")) S->fail_launch_at = std::strtoull(t, nullptr, 10);
  hipError_t e;
  if ((e = hipMalloc(&S->dev_base, c.arena_bytes))) return fail(GRIM_ENOMEM, "device arena", e);
  S->dev_arena = serve::Arena(c.arena_bytes);
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&S->host_base), c.host_arena_bytes, hipHostMallocDefault)))
    return fail(GRIM_ENOMEM, "host arena", e);
  S->host_arena = serve::Arena(c.host_arena_bytes);
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&S->status_pinned), c.max_inflight * sizeof(uint32_t),
                         hipHostMallocDefault)))
    return fail(GRIM_ENOMEM, "status words", e);
  for (uint32_t i = 0; i < c.max_inflight; ++i) S->status_free.push_back(c.max_inflight - 1 - i);
  if ((e = hipStreamCreateWithFlags(&S->prep, hipStreamNonBlocking))) return fail(GRIM_EDEVICE, "stream", e);
  S->streams.resize(c.n_streams);
  for (auto& s : S->streams)
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking))) return fail(GRIM_EDEVICE, "stream", e);
  const uint32_t n_slots = c.policy == GRIM_SERVE_PLAIN ? 2 : 2 * c.n_streams;
  const uint64_t desc_cap = std::max<uint64_t>(c.max_batch_reads, c.max_request_reads);
  S->slots.resize(n_slots);
  for (auto& L : S->slots) {
    if ((e = hipMalloc(reinterpret_cast<void**>(&L.desc), desc_cap * sizeof(ReadDesc))))
      return fail(GRIM_ENOMEM, "launch descriptors", e);
    if ((e = hipMalloc(reinterpret_cast<void**>(&L.order), desc_cap * sizeof(uint32_t))))
      return fail(GRIM_ENOMEM, "launch order", e);
    if ((e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming))) return fail(GRIM_EDEVICE, "event", e);
  }
  grim_server* raw = S.release();
  raw->thread = std::thread(scheduler, raw);
  *out = raw;
  return GRIM_OK;
}

extern "C" int grim_serve_submit(grim_server* S, const grim_reads* rd, uint64_t* ticket) {
  clear_error();
  if (!S || !rd || !ticket) return set_error(GRIM_EINVAL, "NULL argument");
  if (rd->on_device > 1) return set_error(GRIM_EINVAL, "reads.on_device must be 0 or 1");
  if (rd->n_reads == 0) return set_error(GRIM_EINVAL, "empty request");
  if (rd->n_reads > S->cfg.max_request_reads) return set_error(GRIM_EINVAL, "request larger than max_request_reads");
  if (!rd->offsets || (rd->n_bases && !rd->bases)) return set_error(GRIM_EINVAL, "NULL read arrays");
  if (rd->flags) return set_error(GRIM_EINVAL, "per-request flags are set in the server config");
  if (!rd->on_device && (rd->offsets[0] != 0 || (uint64_t)rd->offsets[rd->n_reads] != rd->n_bases))
    return set_error(GRIM_EINVAL, "offsets must run from 0 to n_bases");
  auto r = std::make_unique<Request>();
  r->n_reads = rd->n_reads;
  r->n_bases = rd->n_bases;
  r->edits_kind = rd->max_edits ? 1u : (rd->err_permille ? 2u : 0u);
  r->err_all = rd->err_permille_all;
  r->fp = serve::footprint(rd->n_reads, rd->n_bases, r->edits_kind != 0, S->idx->W,
                           token_capacity(rd->n_bases, rd->n_reads), sizeof(ReadDesc));
  const uint64_t host_bytes = r->fp.off_edits + (r->edits_kind ? serve::up256(rd->n_reads * 2) : 0);
  const uint16_t* edits = r->edits_kind == 1 ? rd->max_edits : rd->err_permille;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return set_error(GRIM_ECANCELED, "server is shutting down");
    if (S->dev_arena.aligned(r->fp.total) > S->dev_arena.capacity()) {
      S->n_rejected++;
      return set_error(GRIM_ENOMEM, "request needs %llu device bytes, more than the server's arena (%llu)",
                       (unsigned long long)r->fp.total, (unsigned long long)S->dev_arena.capacity());
    }
    if (host_bytes > S->host_arena.capacity()) {
      S->n_rejected++;
      return set_error(GRIM_ENOMEM, "request larger than the host staging arena");
    }
    if (!S->fatal.empty()) return set_error(GRIM_EDEVICE, "server stopped: %s", S->fatal.c_str());
    if (!S->host_arena.alloc(host_bytes, &r->host_off))
      return set_error(GRIM_EAGAIN, "host staging is full; retry when requests complete");
    r->host_held = true;
  }
  // the request's host block is held; copy the reads in without the lock
  uint8_t* h = S->host_base + r->host_off;
  int rc = GRIM_OK;
  if (!rd->on_device) {
    std::memcpy(h + r->fp.off_bases, rd->bases, rd->n_bases);
    std::memcpy(h + r->fp.off_offsets, rd->offsets, (rd->n_reads + 1) * 8);
    if (r->edits_kind) std::memcpy(h + r->fp.off_edits, edits, rd->n_reads * 2);
  } else {
    // device reads: synchronous copies into the pinned block (the caller's
    // arrays must be ready on the device; they are not used after the call)
    DeviceGuard dg(S->device);
    hipError_t e = hipMemcpy(h + r->fp.off_offsets, rd->offsets, (rd->n_reads + 1) * 8, hipMemcpyDeviceToHost);
    const int64_t* offs = reinterpret_cast<const int64_t*>(h + r->fp.off_offsets);
    if (e == hipSuccess && (offs[0] != 0 || (uint64_t)offs[rd->n_reads] != rd->n_bases)) {
      rc = set_error(GRIM_EINVAL, "offsets must run from 0 to n_bases");
    } else {
      if (e == hipSuccess && rd->n_bases)
        e = hipMemcpy(h + r->fp.off_bases, rd->bases, rd->n_bases, hipMemcpyDeviceToHost);
      if (e == hipSuccess && r->edits_kind)
        e = hipMemcpy(h + r->fp.off_edits, edits, rd->n_reads * 2, hipMemcpyDeviceToHost);
      if (e != hipSuccess) rc = set_error(GRIM_EDEVICE, "copy of device reads failed: %s", hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (rc == GRIM_OK && S->stop) rc = set_error(GRIM_ECANCELED, "server is shutting down");
  if (rc != GRIM_OK) {
    S->host_arena.release(r->host_off);
    return rc;
  }
  r->ticket = S->next_ticket++;
  r->t_submit = Clock::now();
  if (!S->have_first) {
    S->have_first = true;
    S->t_first_submit = r->t_submit;
  }
  *ticket = r->ticket;
  S->queue.push_back(r->ticket);
  S->reqs[r->ticket] = std::move(r);
  S->n_submitted++;
  S->cv_work.notify_one();
  return GRIM_OK;
}

extern "C" int grim_serve_poll(grim_server* S, uint64_t ticket, grim_result* out) {
  clear_error();
  if (!S || !out) return set_error(GRIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(GRIM_EINVAL, "unknown ticket");
  const Request& r = *it->second;
  if (r.state == RState::Queued || r.state == RState::Prepping || r.state == RState::Active) {
    std::memset(out, 0, sizeof *out);
    out->ticket = ticket;
    out->status = GRIM_EAGAIN;
    return GRIM_EAGAIN;
  }
  const int st = fill_result(S, r, out);
  if (st != GRIM_OK) set_error(st, "request %llu ended with status %d", (unsigned long long)ticket, st);
  return st;
}

extern "C" int grim_serve_wait(grim_server* S, uint64_t ticket, int timeout_ms, grim_result* out) {
  clear_error();
  if (!S || !out) return set_error(GRIM_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(GRIM_EINVAL, "unknown ticket");
  Request* r = it->second.get();
  auto pending = [&] {
    return r->state == RState::Queued || r->state == RState::Prepping || r->state == RState::Active;
  };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, [&] { return !pending(); });
  } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !pending(); })) {
    std::memset(out, 0, sizeof *out);
    out->ticket = ticket;
    out->status = GRIM_ETIMEDOUT;
    return set_error(GRIM_ETIMEDOUT, "request %llu not done after %d ms", (unsigned long long)ticket, timeout_ms);
  }
  const int st = fill_result(S, *r, out);
  if (st != GRIM_OK) set_error(st, "request %llu ended with status %d", (unsigned long long)ticket, st);
  return st;
}

extern "C" int grim_serve_release(grim_server* S, uint64_t ticket) {
  clear_error();
  if (!S) return set_error(GRIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(GRIM_EINVAL, "unknown ticket");
  Request& r = *it->second;
  if (r.state == RState::Queued || r.state == RState::Prepping || r.state == RState::Active)
    return set_error(GRIM_EAGAIN, "request %llu is still being served", (unsigned long long)ticket);
  if (r.dev_held) {
    S->dev_arena.release(r.dev_off);
    r.dev_held = false;
  }
  S->reqs.erase(it);
  S->cv_work.notify_one();
  return GRIM_OK;
}

extern "C" int grim_serve_cancel(grim_server* S, uint64_t ticket) {
  clear_error();
  if (!S) return set_error(GRIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(GRIM_EINVAL, "unknown ticket");
  Request& r = *it->second;
  if (r.state == RState::Queued) {
    finish(S, r, RState::Canceled, GRIM_ECANCELED);
  } else if (r.state == RState::Prepping) {
    r.cancel_requested = true;
  } else if (r.state == RState::Active) {
    r.cancel_requested = true;
    S->former.remove(ticket);
    if (r.launches_in_flight == 0) {
      S->admitted--;
      finish(S, r, RState::Canceled, GRIM_ECANCELED);
    }
  }
  S->cv_work.notify_one();
  return GRIM_OK;
}

extern "C" int grim_serve_stats(grim_server* S, grim_serve_stats_t* out) {
  clear_error();
  if (!S || !out) return set_error(GRIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = S->n_submitted;
  out->completed = S->n_completed;
  out->failed = S->n_failed;
  out->rejected = S->n_rejected;
  out->canceled = S->n_canceled;
  out->reads_completed = S->reads_completed;
  out->launches = S->launches;
  out->shared_launches = S->shared_launches;
  out->max_requests_per_launch = S->max_reqs_per_launch;
  out->peak_device_bytes = S->peak_dev;
  out->arena_bytes = S->cfg.arena_bytes;
  out->p50_ms = serve::nearest_rank(S->latencies, 50.0);
  out->p99_ms = serve::nearest_rank(S->latencies, 99.0);
  out->max_ms = S->latencies.empty() ? 0.0 : *std::max_element(S->latencies.begin(), S->latencies.end());
  double sum = 0;
  for (double v : S->latencies) sum += v;
  out->mean_ms = S->latencies.empty() ? 0.0 : sum / (double)S->latencies.size();
  const double span = S->have_first && S->n_completed ? ms_since(S->t_first_submit, S->t_last_done) : 0.0;
  out->reads_per_s = span > 0 ? (double)S->reads_completed / (span * 1e-3) : 0.0;
  out->queued = (uint32_t)S->queue.size();
  out->admitted = S->admitted;
  return GRIM_OK;
}

extern "C" int grim_serve_reset_stats(grim_server* S) {
  clear_error();
  if (!S) return set_error(GRIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  S->n_submitted = S->n_completed = S->n_failed = S->n_rejected = S->n_canceled = S->reads_completed = 0;
  S->launches = S->shared_launches = S->max_reqs_per_launch = 0;
  S->peak_dev = S->dev_arena.used();
  S->latencies.clear();
  S->have_first = false;
  return GRIM_OK;
}

extern "C" void grim_serve_destroy(grim_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // queued requests are cancelled; admitted ones drain
    for (uint64_t t : S->queue) {
      Request& r = *S->reqs[t];
      if (r.state == RState::Queued) finish(S, r, RState::Canceled, GRIM_ECANCELED);
    }
    S->queue.clear();
    S->cv_work.notify_all();
  }
  if (S->thread.joinable()) S->thread.join();
  DeviceGuard dg(S->device);
  for (auto s : S->streams) (void)hipStreamSynchronize(s);
  if (S->prep) (void)hipStreamSynchronize(S->prep);
  release_all(S);
  delete S;
}
