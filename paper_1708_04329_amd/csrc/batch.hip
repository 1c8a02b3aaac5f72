// Batching layer: launch-shape autotuning and a graph-captured steady-state
// loop. Neither changes the arithmetic: both drive the same tokenize / scan /
// candidate kernels as grim_filter_scan and grim_filter_candidates.
//
//  * grim_tune times every launch shape of one mode (all-bins: threads per
//    workgroup, reads per LDS batch, words per lane; candidates: wavefronts
//    per workgroup, per-read grid or persistent work-queue grid and its size)
//    on a sample of reads, keeps the fastest on the index, and caches it in a
//    text file (GRIM_TUNE_CACHE) keyed by architecture, mode, q and size class.
//  * grim_batcher owns pinned host buffers, device buffers and one
//    instantiated hipGraph per slot holding the batch's kernel sequence
//    (zero status -> tokenize -> filter). Batch sizes travel in a device
//    parameter block, so one capture serves every batch up to the slot's
//    capacity. Each submit is stream-ordered on the slot's stream: exact-size
//    H2D copies, the graph launch, exact-size D2H copies. Two slots on two
//    streams overlap one batch's transfers with the other's kernels.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "grim_internal.h"

namespace grim {

int status_to_error(uint32_t st);

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

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(uint64_t n) { return hipMalloc(reinterpret_cast<void**>(&p), std::max<uint64_t>(n, 1) * sizeof(T)); }
};

// ------------------------------ tune cache --------------------------------
std::string tune_key(const grim_index* idx, uint32_t mode, uint64_t n_reads, uint64_t n_bases, uint64_t n_cand) {
  char buf[160];
  const int nb_log2 = idx->nb ? (int)std::floor(std::log2((double)idx->nb)) : 0;
  const uint64_t mean_len = n_reads ? n_bases / n_reads : 0;
  const int cand_log2 = (n_reads && n_cand) ? (int)std::floor(std::log2((double)n_cand / n_reads + 1.0)) : 0;
  if (mode == GRIM_MODE_SCAN)
    std::snprintf(buf, sizeof buf, "gfx950/scan/q%u/nb2^%d/len%llu", idx->q, nb_log2,
                  (unsigned long long)(mean_len / 25 * 25));
  else
    std::snprintf(buf, sizeof buf, "gfx950/cand/q%u/len%llu/cand2^%d", idx->q,
                  (unsigned long long)(mean_len / 25 * 25), cand_log2);
  return buf;
}

void cache_store(const std::string& key, const grim_tune_result& r) {
  const char* path = std::getenv("GRIM_TUNE_CACHE");
  if (!path || !*path) return;
  std::vector<std::string> lines;
  {
    std::ifstream in(path);
    std::string l;
    while (std::getline(in, l))
      if (l.rfind(key + " ", 0) != 0) lines.push_back(l);
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s %u %u %u %u %u %u %u %.6f", key.c_str(), r.threads, r.reads_per_chunk,
                r.lane_words, r.cand_waves, r.cand_persistent, r.cand_groups_per_cu, r.cand_coop, r.best_ms);
  lines.push_back(buf);
  std::ofstream out(path, std::ios::trunc);
  for (auto& l : lines) out << l << "\n";
}

bool cache_load(const std::string& key, grim_tune_result* r) {
  const char* path = std::getenv("GRIM_TUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream in(path);
  std::string l;
  while (std::getline(in, l)) {
    if (l.rfind(key + " ", 0) != 0) continue;
    std::istringstream ss(l.substr(key.size() + 1));
    grim_tune_result t{};
    if (ss >> t.threads >> t.reads_per_chunk >> t.lane_words >> t.cand_waves >> t.cand_persistent >>
        t.cand_groups_per_cu >> t.cand_coop >> t.best_ms) {
      *r = t;
      return true;
    }
  }
  return false;
}

void to_result(const grim_index* idx, uint32_t mode, grim_tune_result* r) {
  std::memset(r, 0, sizeof *r);
  r->mode = mode;
  r->threads = (uint32_t)idx->scan_cfg.threads;
  r->reads_per_chunk = (uint32_t)idx->scan_cfg.reads_per_chunk;
  r->lane_words = (uint32_t)idx->scan_cfg.lane_words;
  r->cand_waves = (uint32_t)idx->cand_cfg.waves;
  r->cand_persistent = (uint32_t)idx->cand_cfg.persistent;
  r->cand_groups_per_cu = (uint32_t)idx->cand_cfg.groups_per_cu;
  r->cand_coop = (uint32_t)idx->cand_cfg.coop;
}

int apply_result(grim_index* idx, const grim_tune_result* r) {
  if (r->mode == GRIM_MODE_SCAN) {
    if (r->threads != 256 && r->threads != 512 && r->threads != 1024)
      return set_error(GRIM_EINVAL, "threads must be 256, 512 or 1024");
    if (r->lane_words != 4 && r->lane_words != 8) return set_error(GRIM_EINVAL, "lane_words must be 4 or 8");
    if (r->reads_per_chunk < 64 || r->reads_per_chunk > (1u << 20))
      return set_error(GRIM_EINVAL, "reads_per_chunk must be in [64, 2^20]");
    idx->scan_cfg.threads = (int)r->threads;
    idx->scan_cfg.reads_per_chunk = (int)r->reads_per_chunk;
    idx->scan_cfg.lane_words = (int)r->lane_words;
    idx->scan_tuned = true;
  } else if (r->mode == GRIM_MODE_CANDIDATES) {
    if (r->cand_waves > 8) return set_error(GRIM_EINVAL, "cand_waves must be in [0, 8]");
    if (r->cand_persistent > 2) return set_error(GRIM_EINVAL, "cand_persistent must be 0, 1 or 2");
    if (r->cand_groups_per_cu < 1 || r->cand_groups_per_cu > 64)
      return set_error(GRIM_EINVAL, "cand_groups_per_cu must be in [1, 64]");
    if (r->cand_coop > 2) return set_error(GRIM_EINVAL, "cand_coop must be 0, 1 or 2");
    idx->cand_cfg.coop = (int)r->cand_coop;
    idx->cand_cfg.waves = (int)r->cand_waves;
    idx->cand_cfg.persistent = (int)r->cand_persistent;
    idx->cand_cfg.groups_per_cu = (int)r->cand_groups_per_cu;
    idx->cand_tuned = true;
  } else {
    return set_error(GRIM_EINVAL, "mode must be GRIM_MODE_SCAN or GRIM_MODE_CANDIDATES");
  }
  return GRIM_OK;
}

}  // namespace

// Called by the filter entry points before their first launch on an index
// that has not been tuned: adopt a cached shape for this size class, if any.
void apply_cached_config(grim_index* idx, uint32_t mode, uint64_t n_reads, uint64_t n_bases, uint64_t n_cand) {
  if ((mode == GRIM_MODE_SCAN && idx->scan_tuned) || (mode == GRIM_MODE_CANDIDATES && idx->cand_tuned)) return;
  grim_tune_result r{};
  if (cache_load(tune_key(idx, mode, n_reads, n_bases, n_cand), &r)) {
    r.mode = mode;
    (void)apply_result(idx, &r);
  }
}

// Shared with api.hip: stage + tokenize a read set into the index workspace.
int prepare_reads(grim_index* idx, const grim_reads* rd, uint32_t max_tokens, uint32_t tok_shift, hipStream_t s,
                  const int64_t** offsets_dev);

}  // namespace grim

using namespace grim;

// ---------------------------------------------------------------------------
// grim_tune
// ---------------------------------------------------------------------------
extern "C" int grim_tune(grim_index* idx, const grim_reads* rd, const int64_t* cand_off, const int32_t* cand_bin,
                         uint64_t n_cand, void* hip_stream, grim_tune_result* out) {
  clear_error();
  if (!idx || !rd || !out) return set_error(GRIM_EINVAL, "NULL argument");
  if (rd->n_reads == 0) return set_error(GRIM_EINVAL, "tuning needs a non-empty sample");
  const uint32_t mode = cand_off ? GRIM_MODE_CANDIDATES : GRIM_MODE_SCAN;
  if (mode == GRIM_MODE_SCAN && !(idx->layout & GRIM_LAYOUT_TM))
    return set_error(GRIM_EINVAL, "index has no token-major layout");
  if (mode == GRIM_MODE_CANDIDATES && !(idx->layout & GRIM_LAYOUT_BM))
    return set_error(GRIM_EINVAL, "index has no bin-major layout");
  if (mode == GRIM_MODE_CANDIDATES && n_cand && !cand_bin) return set_error(GRIM_EINVAL, "cand_bin is NULL");
  std::lock_guard<std::mutex> lk(idx->mu);
  DeviceGuard dg(idx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int64_t* offs = nullptr;
  int rc = prepare_reads(idx, rd, 65535u, mode == GRIM_MODE_SCAN ? scan_token_shift(idx->q) : 0u, s, &offs);
  if (rc) return rc;
  GRIM_HIP_TRY(hipMemcpyAsync(idx->ws.status_host, idx->ws.status, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  rc = status_to_error(idx->ws.status_host[0] & ~(uint32_t)(ST_BAD_BIN | ST_BAD_CAND_OFF));
  if (rc) return rc;

  hipEvent_t e0, e1;
  GRIM_HIP_TRY(hipEventCreate(&e0));
  GRIM_HIP_TRY(hipEventCreate(&e1));
  auto cleanup = [&]() {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  };
  grim_tune_result best{};
  best.best_ms = 1e30;
  uint32_t tried = 0;
  double default_ms = 0.0;
  // time one launch shape: one warm launch, then the best of two
  auto time_it = [&](auto launch) -> double {
    if (launch() != hipSuccess) return -1.0;
    double bestt = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess)
        return -1.0;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
      bestt = std::min(bestt, (double)ms);
    }
    return bestt;
  };

  if (mode == GRIM_MODE_SCAN) {
    DevBuf<uint32_t> mask;
    if (mask.alloc(rd->n_reads * idx->W) != hipSuccess) {
      cleanup();
      return set_error(GRIM_ENOMEM, "tuning output buffer");
    }
    ScanArgs a{};
    a.tm = idx->tm;
    a.row_words = idx->row_words;
    a.R4 = idx->R4;
    a.q = idx->q;
    a.nb = idx->nb;
    a.W = idx->W;
    a.tokens = idx->ws.tokens;
    a.offsets = offs;
    a.thr = idx->ws.thr;
    a.n_reads = rd->n_reads;
    a.mask_out = mask.p;
    a.status = idx->ws.status;
    const int threads[] = {512, 1024};
    const int chunks[] = {1024, 2048, 4096, 8192};
    const int lws[] = {4, 8};
    for (int lw : lws)
      for (int nt : threads)
        for (int ch : chunks) {
          if (lw == 8 && nt == 1024) continue;  // does not fit the register file
          ScanConfig c;
          c.threads = nt;
          c.reads_per_chunk = ch;
          c.lane_words = lw;
          const double ms = time_it([&] { return launch_scan_allbins(a, c, s); });
          if (ms < 0) continue;
          ++tried;
          if (nt == 1024 && ch == 4096 && lw == 4) default_ms = ms;
          if (ms < best.best_ms) {
            best.best_ms = ms;
            best.threads = (uint32_t)nt;
            best.reads_per_chunk = (uint32_t)ch;
            best.lane_words = (uint32_t)lw;
          }
        }
    if (default_ms > 0 && best.best_ms > 0.95 * default_ms) {  // within noise of the default: keep it
      best.best_ms = default_ms;
      best.threads = 1024;
      best.reads_per_chunk = 4096;
      best.lane_words = 4;
    }
    best.cand_waves = (uint32_t)idx->cand_cfg.waves;
    best.cand_persistent = (uint32_t)idx->cand_cfg.persistent;
    best.cand_groups_per_cu = (uint32_t)idx->cand_cfg.groups_per_cu;
    best.cand_coop = (uint32_t)idx->cand_cfg.coop;
  } else {
    DevBuf<uint16_t> cnt;
    DevBuf<uint8_t> pas;
    if (cnt.alloc(n_cand) != hipSuccess || pas.alloc(n_cand) != hipSuccess) {
      cleanup();
      return set_error(GRIM_ENOMEM, "tuning output buffers");
    }
    CandArgs a{};
    a.bm = idx->bm;
    a.vec_words = idx->vec_words;
    a.R4 = idx->R4;
    a.q = idx->q;
    a.nb = idx->nb;
    a.tokens = idx->ws.tokens;
    a.offsets = offs;
    a.thr = idx->ws.thr;
    a.n_reads = rd->n_reads;
    a.cand_off = cand_off;
    a.cand_bin = cand_bin;
    a.n_cand = n_cand;
    a.count_out = cnt.p;
    a.pass_out = pas.p;
    a.status = idx->ws.status;
    a.work = idx->ws.status + 4;
    const int waves[] = {1, 2, 4, 8};
    const CandConfig dflt = default_cand_config(idx->vec_words);
    // lane layouts: one lane per pair; groups of lanes per pair (q >= 5); four reads per wavefront (q = 5)
    const int max_coop = idx->vec_words == 32 ? 2 : (idx->vec_words > 32 && idx->vec_words <= 512 ? 1 : 0);
    for (int coop = 0; coop <= max_coop; ++coop)
      for (int nw : waves)
        for (int pers = 0; pers <= 1; ++pers)
          for (int gpc : {2, 4, 8, 16}) {
            if (!pers && gpc != 2) continue;
            CandConfig c;
            c.waves = nw;
            c.persistent = pers;
            c.groups_per_cu = gpc;
            c.coop = coop;
            const double ms = time_it([&] { return launch_scan_candidates(a, c, s); });
            if (ms < 0) continue;
            ++tried;
            // the shape an untuned index uses (default_cand_config)
            if (coop == dflt.coop && (dflt.waves == 0 || nw == dflt.waves) && pers == dflt.persistent &&
                gpc == dflt.groups_per_cu && (dflt.waves != 0 || nw == 8))
              default_ms = ms;
            if (ms < best.best_ms) {
              best.best_ms = ms;
              best.cand_waves = (uint32_t)nw;
              best.cand_persistent = (uint32_t)pers;
              best.cand_groups_per_cu = (uint32_t)gpc;
              best.cand_coop = (uint32_t)coop;
            }
          }
    // a shape that beats the default by under 5% on the sample is noise more
    // often than not (short samples are dominated by launch overhead): keep the default
    if (default_ms > 0 && best.best_ms > 0.95 * default_ms) {
      best.best_ms = default_ms;
      best.cand_waves = (uint32_t)dflt.waves;
      best.cand_persistent = (uint32_t)dflt.persistent;
      best.cand_groups_per_cu = (uint32_t)dflt.groups_per_cu;
      best.cand_coop = (uint32_t)dflt.coop;
    }
    best.threads = (uint32_t)idx->scan_cfg.threads;
    best.reads_per_chunk = (uint32_t)idx->scan_cfg.reads_per_chunk;
    best.lane_words = (uint32_t)idx->scan_cfg.lane_words;
  }
  cleanup();
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  // the candidate kernel may have flagged bad bins or offsets in the sample
  GRIM_HIP_TRY(hipMemcpy(idx->ws.status_host, idx->ws.status, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost));
  rc = status_to_error(idx->ws.status_host[0]);
  if (rc) return rc;
  if (tried == 0) return set_error(GRIM_EDEVICE, "no launch shape ran");
  best.mode = mode;
  best.n_tried = tried;
  best.default_ms = default_ms;
  rc = apply_result(idx, &best);
  if (rc) return rc;
  cache_store(tune_key(idx, mode, rd->n_reads, rd->n_bases, n_cand), best);
  *out = best;
  return GRIM_OK;
}

extern "C" int grim_index_get_config(const grim_index* idx, uint32_t mode, grim_tune_result* out) {
  clear_error();
  if (!idx || !out) return set_error(GRIM_EINVAL, "NULL argument");
  if (mode != GRIM_MODE_SCAN && mode != GRIM_MODE_CANDIDATES) return set_error(GRIM_EINVAL, "bad mode");
  to_result(idx, mode, out);
  return GRIM_OK;
}

extern "C" int grim_index_set_config(grim_index* idx, const grim_tune_result* cfg) {
  clear_error();
  if (!idx || !cfg) return set_error(GRIM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(idx->mu);
  return apply_result(idx, cfg);
}

// ---------------------------------------------------------------------------
// grim_batcher: graph-captured steady-state loop
// ---------------------------------------------------------------------------
struct grim_batch_slot {
  hipStream_t stream = nullptr;
  // pinned host side
  uint8_t* h_bases = nullptr;
  int64_t* h_offsets = nullptr;
  uint16_t* h_edits = nullptr;
  int64_t* h_cand_off = nullptr;
  int32_t* h_cand_bin = nullptr;
  uint16_t* h_count = nullptr;
  uint8_t* h_pass = nullptr;
  DynSizes* h_dyn = nullptr;
  uint32_t* h_status = nullptr;
  // device side
  uint8_t* d_bases = nullptr;
  int64_t* d_offsets = nullptr;
  uint16_t* d_edits = nullptr;
  int64_t* d_cand_off = nullptr;
  int32_t* d_cand_bin = nullptr;
  uint16_t* d_count = nullptr;
  uint8_t* d_pass = nullptr;
  uint32_t* d_mask = nullptr;
  uint32_t* d_tokens = nullptr;
  int32_t* d_thr = nullptr;
  uint32_t* d_order = nullptr;
  uint32_t* d_hist = nullptr;
  DynSizes* d_dyn = nullptr;
  uint32_t* d_status = nullptr;
  // the captured kernel sequence
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool pending = false;
};

struct grim_batcher {
  const grim_index* idx = nullptr;
  uint32_t mode = 0;
  uint64_t max_reads = 0, max_bases = 0, max_cand = 0;
  uint32_t edits_kind = 0;  // GRIM_BATCH_EDITS_*
  uint32_t err_permille_all = 0;
  uint32_t flags = 0;
  grim_batch_slot slot[2];
};

namespace {

void free_slot(grim_batch_slot& s) {
  if (s.exec) (void)hipGraphExecDestroy(s.exec);
  if (s.graph) (void)hipGraphDestroy(s.graph);
  for (void* p : {(void*)s.h_bases, (void*)s.h_offsets, (void*)s.h_edits, (void*)s.h_cand_off, (void*)s.h_cand_bin,
                  (void*)s.h_count, (void*)s.h_pass, (void*)s.h_dyn, (void*)s.h_status})
    if (p) (void)hipHostFree(p);
  for (void* p : {(void*)s.d_bases, (void*)s.d_offsets, (void*)s.d_edits, (void*)s.d_cand_off, (void*)s.d_cand_bin,
                  (void*)s.d_count, (void*)s.d_pass, (void*)s.d_mask, (void*)s.d_tokens, (void*)s.d_thr,
                  (void*)s.d_order, (void*)s.d_hist, (void*)s.d_dyn, (void*)s.d_status})
    if (p) (void)hipFree(p);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = grim_batch_slot{};
}

template <typename T>
hipError_t host_alloc(T** p, uint64_t n) {
  return hipHostMalloc(reinterpret_cast<void**>(p), std::max<uint64_t>(n, 1) * sizeof(T), hipHostMallocDefault);
}
template <typename T>
hipError_t dev_alloc(T** p, uint64_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<uint64_t>(n, 1) * sizeof(T));
}

int build_slot(grim_batcher* b, grim_batch_slot& s) {
  const grim_index* idx = b->idx;
  const bool cand = b->mode == GRIM_MODE_CANDIDATES;
  GRIM_HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
  GRIM_HIP_TRY(host_alloc(&s.h_bases, b->max_bases));
  GRIM_HIP_TRY(host_alloc(&s.h_offsets, b->max_reads + 1));
  GRIM_HIP_TRY(host_alloc(&s.h_dyn, 1));
  GRIM_HIP_TRY(host_alloc(&s.h_status, 8));
  GRIM_HIP_TRY(dev_alloc(&s.d_bases, b->max_bases));
  GRIM_HIP_TRY(dev_alloc(&s.d_offsets, b->max_reads + 1));
  GRIM_HIP_TRY(dev_alloc(&s.d_dyn, 1));
  GRIM_HIP_TRY(dev_alloc(&s.d_status, 8));
  GRIM_HIP_TRY(dev_alloc(&s.d_tokens, token_capacity(b->max_bases, b->max_reads)));
  GRIM_HIP_TRY(dev_alloc(&s.d_thr, b->max_reads + 1));
  if (b->edits_kind != GRIM_BATCH_EDITS_NONE) {
    GRIM_HIP_TRY(host_alloc(&s.h_edits, b->max_reads));
    GRIM_HIP_TRY(dev_alloc(&s.d_edits, b->max_reads));
  }
  if (cand) {
    GRIM_HIP_TRY(host_alloc(&s.h_cand_off, b->max_reads + 1));
    GRIM_HIP_TRY(host_alloc(&s.h_cand_bin, b->max_cand));
    GRIM_HIP_TRY(host_alloc(&s.h_count, b->max_cand));
    GRIM_HIP_TRY(host_alloc(&s.h_pass, b->max_cand));
    GRIM_HIP_TRY(dev_alloc(&s.d_cand_off, b->max_reads + 1));
    GRIM_HIP_TRY(dev_alloc(&s.d_cand_bin, b->max_cand));
    GRIM_HIP_TRY(dev_alloc(&s.d_count, b->max_cand));
    GRIM_HIP_TRY(dev_alloc(&s.d_pass, b->max_cand));
  } else {
    GRIM_HIP_TRY(dev_alloc(&s.d_mask, b->max_reads * idx->W));
    GRIM_HIP_TRY(dev_alloc(&s.d_order, b->max_reads));
    GRIM_HIP_TRY(dev_alloc(&s.d_hist, length_order_scratch_words()));
  }
  std::memset(s.h_dyn, 0, sizeof(DynSizes));

  // kernels: captured from a stream into a child graph
  hipGraph_t kernels = nullptr;
  GRIM_HIP_TRY(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_zero_words(s.d_status, 8, s.stream);
  if (e == hipSuccess) {
    TokArgs t{};
    t.dyn = s.d_dyn;
    t.bases = s.d_bases;
    t.offsets = s.d_offsets;
    t.n_reads = b->max_reads;
    t.n_bases = b->max_bases;
    t.max_edits = b->edits_kind == GRIM_BATCH_EDITS_MAX ? s.d_edits : nullptr;
    t.err_pm = b->edits_kind == GRIM_BATCH_EDITS_ERR ? s.d_edits : nullptr;
    t.err_pm_all = b->err_permille_all;
    t.q = idx->q;
    t.overlap = idx->O;
    t.flags = b->flags;
    t.max_tokens = 65535u;
    t.tok_shift = cand ? 0u : scan_token_shift(idx->q);
    t.short_pad = cand ? 1u : 0u;
    t.pair_order = !cand && t.tok_shift == 7 ? 1u : 0u;
    t.tokens = s.d_tokens;
    t.thr = s.d_thr;
    t.status = s.d_status;
    e = launch_tokenize(t, s.stream);
  }
  if (e == hipSuccess) {
    if (cand) {
      CandArgs a{};
      a.dyn = s.d_dyn;
      a.work = s.d_status + 4;
      a.bm = idx->bm;
      a.vec_words = idx->vec_words;
      a.R4 = idx->R4;
      a.q = idx->q;
      a.nb = idx->nb;
      a.tokens = s.d_tokens;
      a.offsets = s.d_offsets;
      a.thr = s.d_thr;
      a.n_reads = b->max_reads;
      a.cand_off = s.d_cand_off;
      a.cand_bin = s.d_cand_bin;
      a.n_cand = b->max_cand;
      a.count_out = s.d_count;
      a.pass_out = s.d_pass;
      a.status = s.d_status;
      e = launch_scan_candidates(a, idx->cand_cfg, s.stream);
    } else {
      ScanArgs a{};
      a.dyn = s.d_dyn;
      a.tm = idx->tm;
      a.row_words = idx->row_words;
      a.R4 = idx->R4;
      a.q = idx->q;
      a.nb = idx->nb;
      a.W = idx->W;
      a.tokens = s.d_tokens;
      a.offsets = s.d_offsets;
      a.thr = s.d_thr;
      a.n_reads = b->max_reads;
      a.mask_out = s.d_mask;
      a.status = s.d_status;
      if (idx->scan_cfg.sort_by_length) {
        e = launch_length_order(s.d_offsets, b->max_reads, idx->q, s.d_dyn, s.d_hist, s.d_order, s.stream);
        a.read_order = s.d_order;
      }
      if (e == hipSuccess) e = launch_scan_allbins(a, idx->scan_cfg, s.stream);
    }
  }
  hipError_t ec = hipStreamEndCapture(s.stream, &kernels);
  if (e != hipSuccess || ec != hipSuccess) {
    if (kernels) (void)hipGraphDestroy(kernels);
    return set_error(GRIM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : ec));
  }
  s.graph = kernels;
  GRIM_HIP_TRY(hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0));
  return GRIM_OK;
}

}  // namespace

extern "C" int grim_batcher_create(const grim_index* idx, uint32_t mode, uint64_t max_reads, uint64_t max_bases,
                                   uint64_t max_cand, uint32_t edits_kind, uint32_t err_permille_all, uint32_t flags,
                                   grim_batcher** out) {
  clear_error();
  if (!idx || !out) return set_error(GRIM_EINVAL, "NULL argument");
  *out = nullptr;
  if (mode != GRIM_MODE_SCAN && mode != GRIM_MODE_CANDIDATES) return set_error(GRIM_EINVAL, "bad mode");
  if (mode == GRIM_MODE_SCAN && !(idx->layout & GRIM_LAYOUT_TM))
    return set_error(GRIM_EINVAL, "index has no token-major layout");
  if (mode == GRIM_MODE_CANDIDATES && !(idx->layout & GRIM_LAYOUT_BM))
    return set_error(GRIM_EINVAL, "index has no bin-major layout");
  if (max_reads == 0 || max_bases == 0 || (mode == GRIM_MODE_CANDIDATES && max_cand == 0))
    return set_error(GRIM_EINVAL, "capacities must be positive");
  if (max_reads > (1ull << 32) || max_bases > (1ull << 40) || max_cand > (1ull << 36))
    return set_error(GRIM_EINVAL, "capacity too large");
  if (edits_kind > GRIM_BATCH_EDITS_ERR) return set_error(GRIM_EINVAL, "bad edits_kind");
  if (flags & ~GRIM_READS_ALLOW_SHORT_OVERLAP) return set_error(GRIM_EINVAL, "unknown flags");
  DeviceGuard dg(idx->device);
  auto* b = new grim_batcher;
  b->idx = idx;
  b->mode = mode;
  b->max_reads = max_reads;
  b->max_bases = max_bases;
  b->max_cand = max_cand;
  b->edits_kind = edits_kind;
  b->err_permille_all = err_permille_all;
  b->flags = flags;
  for (auto& s : b->slot) {
    const int rc = build_slot(b, s);
    if (rc) {
      for (auto& t : b->slot) free_slot(t);
      delete b;
      return rc;
    }
  }
  *out = b;
  return GRIM_OK;
}

extern "C" int grim_batcher_buffers(grim_batcher* b, uint32_t slot, grim_batch_buffers* out) {
  clear_error();
  if (!b || !out || slot > 1) return set_error(GRIM_EINVAL, "bad argument");
  grim_batch_slot& s = b->slot[slot];
  std::memset(out, 0, sizeof *out);
  out->bases = s.h_bases;
  out->offsets = s.h_offsets;
  out->edits = s.h_edits;
  out->cand_off = s.h_cand_off;
  out->cand_bin = s.h_cand_bin;
  out->count_out = s.h_count;
  out->pass_out = s.h_pass;
  out->mask_out = s.d_mask;
  return GRIM_OK;
}

extern "C" int grim_batcher_submit(grim_batcher* b, uint32_t slot, uint64_t n_reads, uint64_t n_bases,
                                   uint64_t n_cand) {
  clear_error();
  if (!b || slot > 1) return set_error(GRIM_EINVAL, "bad argument");
  grim_batch_slot& s = b->slot[slot];
  if (s.pending) return set_error(GRIM_EINVAL, "slot %u still has a batch in flight", slot);
  if (n_reads > b->max_reads || n_bases > b->max_bases || n_cand > b->max_cand)
    return set_error(GRIM_EINVAL, "batch larger than the batcher's capacity");
  if (s.h_offsets[0] != 0 && n_reads) return set_error(GRIM_EINVAL, "offsets[0] must be 0");
  if (b->mode == GRIM_MODE_CANDIDATES && n_reads && (s.h_cand_off[0] != 0 || (uint64_t)s.h_cand_off[n_reads] != n_cand))
    return set_error(GRIM_EINVAL, "cand_off must run from 0 to n_cand");
  DeviceGuard dg(b->idx->device);
  s.h_dyn->n_reads = n_reads;
  s.h_dyn->n_bases = n_bases;
  s.h_dyn->n_cand = n_cand;
  const hipMemcpyKind h2d = hipMemcpyHostToDevice, d2h = hipMemcpyDeviceToHost;
  GRIM_HIP_TRY(hipMemcpyAsync(s.d_dyn, s.h_dyn, sizeof(DynSizes), h2d, s.stream));
  if (n_bases) GRIM_HIP_TRY(hipMemcpyAsync(s.d_bases, s.h_bases, n_bases, h2d, s.stream));
  GRIM_HIP_TRY(hipMemcpyAsync(s.d_offsets, s.h_offsets, (n_reads + 1) * 8, h2d, s.stream));
  if (s.d_edits && n_reads) GRIM_HIP_TRY(hipMemcpyAsync(s.d_edits, s.h_edits, n_reads * 2, h2d, s.stream));
  if (b->mode == GRIM_MODE_CANDIDATES) {
    GRIM_HIP_TRY(hipMemcpyAsync(s.d_cand_off, s.h_cand_off, (n_reads + 1) * 8, h2d, s.stream));
    if (n_cand) GRIM_HIP_TRY(hipMemcpyAsync(s.d_cand_bin, s.h_cand_bin, n_cand * 4, h2d, s.stream));
  }
  GRIM_HIP_TRY(hipGraphLaunch(s.exec, s.stream));
  GRIM_HIP_TRY(hipMemcpyAsync(s.h_status, s.d_status, 8 * sizeof(uint32_t), d2h, s.stream));
  if (b->mode == GRIM_MODE_CANDIDATES && n_cand) {
    GRIM_HIP_TRY(hipMemcpyAsync(s.h_count, s.d_count, n_cand * 2, d2h, s.stream));
    GRIM_HIP_TRY(hipMemcpyAsync(s.h_pass, s.d_pass, n_cand, d2h, s.stream));
  }
  s.pending = true;
  return GRIM_OK;
}

extern "C" int grim_batcher_wait(grim_batcher* b, uint32_t slot) {
  clear_error();
  if (!b || slot > 1) return set_error(GRIM_EINVAL, "bad argument");
  grim_batch_slot& s = b->slot[slot];
  if (!s.pending) return GRIM_OK;
  DeviceGuard dg(b->idx->device);
  s.pending = false;
  GRIM_HIP_TRY(hipStreamSynchronize(s.stream));
  return status_to_error(s.h_status[0]);
}

extern "C" void* grim_batcher_stream(grim_batcher* b, uint32_t slot) {
  if (!b || slot > 1) return nullptr;
  return b->slot[slot].stream;
}

extern "C" void grim_batcher_free(grim_batcher* b) {
  if (!b) return;
  DeviceGuard dg(b->idx->device);
  for (auto& s : b->slot) {
    if (s.pending && s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  delete b;
}
