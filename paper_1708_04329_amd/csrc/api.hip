// Entry points of libgrim (declared in include/grim.h): argument checks,
// device memory, stream ordering and error reporting around the kernels.

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <vector>

#include "grim_internal.h"

namespace grim {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}
const char* last_error() { return t_err.c_str(); }
void clear_error() { t_err.clear(); }

int status_to_error(uint32_t st) {
  if (st == 0) return GRIM_OK;
  if (st & ST_BAD_LENGTH) return set_error(GRIM_EINVAL, "a read is shorter than q or its offsets are out of range");
  if (st & ST_TOO_LONG) return set_error(GRIM_EINVAL, "a read has more than 65535 tokens");
  if (st & ST_COUNT_U8) return set_error(GRIM_EINVAL, "uint8 counts need reads of at most 255 tokens");
  if (st & ST_BAD_CAND_OFF) return set_error(GRIM_EINVAL, "candidate offsets out of order or out of range");
  if (st & ST_BAD_BIN) return set_error(GRIM_EINVAL, "a candidate bin is outside [0, n_bins)");
  if (st & ST_VERIFY_LONG) return set_error(GRIM_EINVAL, "a read to verify is longer than %u bases", kVerifyMaxLen);
  if (st & ST_OVERLAP)
    return set_error(GRIM_EOVERLAP, "a read is not covered by the bin overlap (O < L + E - q)");
  return set_error(GRIM_EINVAL, "invalid input (status 0x%x)", st);
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
static std::atomic<int> g_prof_on{0};
static std::mutex g_prof_mu;
static grim_kernel_time g_prof[PROF_N];

bool profiling() { return g_prof_on.load(std::memory_order_relaxed) != 0; }

void ProfSpan::start(hipStream_t s) {
  if (!profiling()) return;
  if (!ev[0] && hipEventCreate(&ev[0]) != hipSuccess) return;
  if (!ev[1] && hipEventCreate(&ev[1]) != hipSuccess) return;
  on = hipEventRecord(ev[0], s) == hipSuccess;
}
void ProfSpan::stop(hipStream_t s) {
  if (on) on = hipEventRecord(ev[1], s) == hipSuccess;
}
void ProfSpan::collect() {
  if (!on) return;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[kind].launches += 1;
    g_prof[kind].total_ms += ms;
    g_prof[kind].last_ms = ms;
  }
  on = false;
}
ProfSpan::~ProfSpan() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
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

int check_device(int dev) {
  hipDeviceProp_t prop;
  GRIM_HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(GRIM_EDEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  return GRIM_OK;
}

template <typename T>
int grow(T** p, uint64_t* cap, uint64_t need) {
  if (*cap >= need && *p) return GRIM_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  uint64_t n = need + need / 4 + 256;
  void* q = nullptr;
  GRIM_HIP_TRY(hipMalloc(&q, n * sizeof(T)));
  *p = static_cast<T*>(q);
  *cap = n;
  return GRIM_OK;
}

int ensure_status(grim_workspace& ws) {
  if (!ws.status) GRIM_HIP_TRY(hipMalloc(&ws.status, 8 * sizeof(uint32_t)));
  if (!ws.status_host) GRIM_HIP_TRY(hipHostMalloc(&ws.status_host, 8 * sizeof(uint32_t), hipHostMallocDefault));
  return GRIM_OK;
}

void free_workspace(grim_workspace& ws) {
  if (ws.tokens) (void)hipFree(ws.tokens);
  if (ws.thr) (void)hipFree(ws.thr);
  if (ws.status) (void)hipFree(ws.status);
  if (ws.status_host) (void)hipHostFree(ws.status_host);
  if (ws.staging) (void)hipFree(ws.staging);
  if (ws.order) (void)hipFree(ws.order);
  if (ws.hist) (void)hipFree(ws.hist);
  if (ws.vbucket) (void)hipFree(ws.vbucket);
  if (ws.vbucket_host) (void)hipHostFree(ws.vbucket_host);
  if (ws.vitem_pair) (void)hipFree(ws.vitem_pair);
  if (ws.vitem_read) (void)hipFree(ws.vitem_read);
  if (ws.vread_sel) (void)hipFree(ws.vread_sel);
  if (ws.vchunk_sum) (void)hipFree(ws.vchunk_sum);
  ws = grim_workspace{};
}

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Device views of a read set (copying host-resident arrays into staging).
struct ReadView {
  const uint8_t* bases;
  const int64_t* offsets;
  const uint16_t* max_edits;
  const uint16_t* err_pm;
};

int stage_reads(grim_index* idx, const grim_reads* rd, hipStream_t s, ReadView* v) {
  if (rd->on_device) {
    *v = {rd->bases, rd->offsets, rd->max_edits, rd->err_permille};
    return GRIM_OK;
  }
  const uint64_t n = rd->n_reads;
  const uint64_t ob = align_up(rd->n_bases, 256);
  const uint64_t oo = ob + align_up((n + 1) * 8, 256);
  const uint64_t oe = oo + (rd->max_edits ? align_up(n * 2, 256) : 0);
  const uint64_t total = oe + (rd->err_permille ? align_up(n * 2, 256) : 0);
  int rc = grow(&idx->ws.staging, &idx->ws.staging_cap, total);
  if (rc) return rc;
  uint8_t* st = idx->ws.staging;
  if (rd->n_bases) GRIM_HIP_TRY(hipMemcpyAsync(st, rd->bases, rd->n_bases, hipMemcpyHostToDevice, s));
  GRIM_HIP_TRY(hipMemcpyAsync(st + ob, rd->offsets, (n + 1) * 8, hipMemcpyHostToDevice, s));
  if (rd->max_edits) GRIM_HIP_TRY(hipMemcpyAsync(st + oo, rd->max_edits, n * 2, hipMemcpyHostToDevice, s));
  if (rd->err_permille) GRIM_HIP_TRY(hipMemcpyAsync(st + oe, rd->err_permille, n * 2, hipMemcpyHostToDevice, s));
  v->bases = st;
  v->offsets = reinterpret_cast<const int64_t*>(st + ob);
  v->max_edits = rd->max_edits ? reinterpret_cast<const uint16_t*>(st + oo) : nullptr;
  v->err_pm = rd->err_permille ? reinterpret_cast<const uint16_t*>(st + oe) : nullptr;
  return GRIM_OK;
}

int check_reads_args(const grim_index* idx, const grim_reads* rd) {
  if (!idx) return set_error(GRIM_EINVAL, "index is NULL");
  if (!rd) return set_error(GRIM_EINVAL, "reads is NULL");
  if (rd->n_reads && !rd->offsets) return set_error(GRIM_EINVAL, "reads.offsets is NULL");
  if (rd->n_bases && !rd->bases) return set_error(GRIM_EINVAL, "reads.bases is NULL");
  if (rd->on_device > 1) return set_error(GRIM_EINVAL, "reads.on_device must be 0 or 1");
  if (rd->flags & ~GRIM_READS_ALLOW_SHORT_OVERLAP) return set_error(GRIM_EINVAL, "unknown reads.flags bits");
  if (rd->n_reads > (1ull << 40)) return set_error(GRIM_EINVAL, "too many reads");
  return GRIM_OK;
}

// Tokenise + thresholds into the index workspace; leaves status zeroed first.
int tokenize_reads(grim_index* idx, const grim_reads* rd, const ReadView& v, uint32_t max_tokens,
                   uint32_t tok_shift, hipStream_t s, ProfSpan& ps) {
  grim_workspace& ws = idx->ws;
  int rc = ensure_status(ws);
  if (rc) return rc;
  rc = grow(&ws.tokens, &ws.tokens_cap, token_capacity(rd->n_bases, rd->n_reads));
  if (rc) return rc;
  rc = grow(&ws.thr, &ws.thr_cap, rd->n_reads + 1);
  if (rc) return rc;
  GRIM_HIP_TRY(hipMemsetAsync(ws.status, 0, 8 * sizeof(uint32_t), s));
  TokArgs a{};
  a.bases = v.bases;
  a.offsets = v.offsets;
  a.n_reads = rd->n_reads;
  a.n_bases = rd->n_bases;
  a.max_edits = v.max_edits;
  a.err_pm = v.err_pm;
  a.err_pm_all = rd->err_permille_all;
  a.q = idx->q;
  a.overlap = idx->O;
  a.flags = rd->flags;
  a.max_tokens = max_tokens;
  a.tok_shift = tok_shift;
  // plain codes (no shift) serve the candidate and verification calls, which
  // read a read's entries only up to its token count; the scans' shifted
  // entries keep the padding their last block reads
  a.short_pad = tok_shift == 0 ? 1u : 0u;
  // 128-byte tile rows: the all-bins scan reads tokens in pair order
  a.pair_order = tok_shift == 7 ? 1u : 0u;
  a.tokens = ws.tokens;
  a.thr = ws.thr;
  a.status = ws.status;
  ps.start(s);
  GRIM_HIP_TRY(launch_tokenize(a, s));
  ps.stop(s);
  return GRIM_OK;
}

}  // namespace

int prepare_reads(grim_index* idx, const grim_reads* rd, uint32_t max_tokens, uint32_t tok_shift, hipStream_t s,
                  const int64_t** offsets_dev) {
  int rc = check_reads_args(idx, rd);
  if (rc) return rc;
  ReadView v;
  rc = stage_reads(idx, rd, s, &v);
  if (rc) return rc;
  ProfSpan pt(PROF_TOKENIZE);
  rc = tokenize_reads(idx, rd, v, max_tokens, tok_shift, s, pt);
  if (rc) return rc;
  *offsets_dev = v.offsets;
  return GRIM_OK;
}

void apply_cached_config(grim_index* idx, uint32_t mode, uint64_t n_reads, uint64_t n_bases, uint64_t n_cand);

namespace {

int finish_status(grim_index* idx, hipStream_t s) {
  grim_workspace& ws = idx->ws;
  GRIM_HIP_TRY(hipMemcpyAsync(ws.status_host, ws.status, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  return status_to_error(ws.status_host[0]);
}

ScanConfig scan_config_from_env(ScanConfig c) {
  if (const char* t = std::getenv("GRIM_SCAN_THREADS")) c.threads = std::atoi(t);
  if (const char* t = std::getenv("GRIM_SCAN_CHUNK")) c.reads_per_chunk = std::atoi(t);
  if (const char* t = std::getenv("GRIM_SCAN_LANE_WORDS")) c.lane_words = std::atoi(t);
  if (c.threads != 256 && c.threads != 512 && c.threads != 1024) c.threads = 1024;
  if (const char* t = std::getenv("GRIM_SCAN_SORT")) c.sort_by_length = std::atoi(t) ? 1 : 0;
  if (c.lane_words != 4 && c.lane_words != 8) c.lane_words = 4;
  if (c.reads_per_chunk < 64) c.reads_per_chunk = 64;
  return c;
}

CandConfig cand_config_from_env(CandConfig c) {
  if (const char* t = std::getenv("GRIM_CAND_WAVES")) c.waves = std::atoi(t);
  if (const char* t = std::getenv("GRIM_CAND_PERSISTENT")) {
    const int v = std::atoi(t);
    c.persistent = v == 2 ? 2 : (v ? 1 : 0);
  }
  if (const char* t = std::getenv("GRIM_CAND_GROUPS_PER_CU")) c.groups_per_cu = std::atoi(t);
  if (const char* t = std::getenv("GRIM_CAND_COOP")) {
    const int v = std::atoi(t);
    c.coop = v == 2 ? 2 : (v ? 1 : 0);
  }
  if (const char* t = std::getenv("GRIM_CAND_PLANES")) c.planes = std::atoi(t) == 16 ? 16 : 8;
  if (c.waves < 0 || c.waves > 8) c.waves = 0;
  if (c.groups_per_cu < 1 || c.groups_per_cu > 64) c.groups_per_cu = 2;
  return c;
}

// ------------------------------ index file ---------------------------------
struct FileHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  uint64_t G;
  uint32_t B, O, q, layout;
  uint64_t nb, W, row_words;
  uint32_t vec_words, reserved;
  uint64_t tm_bytes, bm_bytes;
  uint64_t checksum;
};
constexpr char kMagic[8] = {'G', 'R', 'I', 'M', 'I', 'D', 'X', '1'};
constexpr uint32_t kFileVersion = 1;

uint64_t fnv1a(uint64_t h, const uint8_t* p, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

int fill_geometry(grim_index* idx, uint64_t G, uint32_t B, uint32_t O, uint32_t q, uint32_t layout) {
  idx->G = G;
  idx->B = B;
  idx->O = O;
  idx->q = q;
  idx->layout = layout;
  idx->nb = (G + B - 1) / B;
  idx->W = (idx->nb + 31) / 32;
  idx->row_words = align_up(idx->W, kTmRowAlign);
  idx->R4 = 1u << (2 * q);
  idx->vec_words = idx->R4 >= 32 ? idx->R4 / 32 : 1;
  idx->tm_bytes = (layout & GRIM_LAYOUT_TM) ? (uint64_t)idx->R4 * idx->row_words * 4 : 0;
  idx->bm_bytes = (layout & GRIM_LAYOUT_BM) ? idx->nb * idx->vec_words * 4 : 0;
  idx->ref_bytes = (layout & GRIM_LAYOUT_REF) ? G : 0;
  idx->cand_cfg = default_cand_config(idx->vec_words);
  return GRIM_OK;
}

int alloc_layouts(grim_index* idx) {
  if (idx->tm_bytes) GRIM_HIP_TRY(hipMalloc(&idx->tm, idx->tm_bytes));
  if (idx->bm_bytes) GRIM_HIP_TRY(hipMalloc(&idx->bm, idx->bm_bytes));
  if (idx->ref_bytes) GRIM_HIP_TRY(hipMalloc(&idx->ref, idx->ref_bytes));
  return GRIM_OK;
}

void destroy(grim_index* idx) {
  if (!idx) return;
  DeviceGuard dg(idx->device);
  if (idx->tm) (void)hipFree(idx->tm);
  if (idx->bm) (void)hipFree(idx->bm);
  if (idx->ref) (void)hipFree(idx->ref);
  free_workspace(idx->ws);
  delete idx;
}

}  // namespace
}  // namespace grim

using namespace grim;

extern "C" {

int grim_abi_version(void) { return GRIM_ABI_VERSION; }

const char* grim_last_error(void) { return grim::last_error(); }

int grim_profile_enable(int on) {
  g_prof_on.store(on ? 1 : 0);
  return GRIM_OK;
}

int grim_profile_read(grim_profile_t* out, int reset) {
  if (!out) return set_error(GRIM_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  out->tokenize = g_prof[PROF_TOKENIZE];
  out->scan = g_prof[PROF_SCAN];
  out->candidates = g_prof[PROF_CAND];
  out->build = g_prof[PROF_BUILD];
  out->verify = g_prof[PROF_VERIFY];
  if (reset)
    for (auto& k : g_prof) k = grim_kernel_time{0, 0.0, 0.0};
  return GRIM_OK;
}

int grim_build_index(const uint8_t* ref, uint64_t ref_len, uint32_t ref_on_device, uint32_t bin_size,
                     uint32_t overlap, uint32_t q, uint32_t layout, void* hip_stream, grim_index** out) {
  clear_error();
  if (!out) return set_error(GRIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ref) return set_error(GRIM_EINVAL, "ref is NULL");
  if (bin_size == 0) return set_error(GRIM_EINVAL, "bin_size must be >= 1");
  if (q < 1 || q > 8) return set_error(GRIM_EINVAL, "q must be in [1, 8]");
  if (q == 8 && (layout & GRIM_LAYOUT_TM))
    return set_error(GRIM_EINVAL, "the token-major layout (all-bins scan) supports q <= 7: a tile of 4^8 + 1 rows "
                                  "does not fit the 160 KB of LDS; use GRIM_LAYOUT_BM (candidate checks) at q = 8");
  if (ref_len < q) return set_error(GRIM_EINVAL, "reference shorter than q");
  if (layout == 0 || (layout & ~(GRIM_LAYOUT_TM | GRIM_LAYOUT_BM | GRIM_LAYOUT_REF)))
    return set_error(GRIM_EINVAL, "layout must be a combination of GRIM_LAYOUT_TM, GRIM_LAYOUT_BM, GRIM_LAYOUT_REF");
  if (ref_on_device > 1) return set_error(GRIM_EINVAL, "ref_on_device must be 0 or 1");
  if ((ref_len + bin_size - 1) / bin_size > (1ull << 31)) return set_error(GRIM_EINVAL, "more than 2^31 bins");
  int dev = 0;
  GRIM_HIP_TRY(hipGetDevice(&dev));
  int rc = check_device(dev);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::unique_ptr<grim_index, void (*)(grim_index*)> idx(new grim_index, destroy);
  idx->device = dev;
  fill_geometry(idx.get(), ref_len, bin_size, overlap, q, layout);
  rc = alloc_layouts(idx.get());
  if (rc) return rc;
  const uint8_t* dref = ref;
  void* staging = nullptr;
  if (!ref_on_device) {
    GRIM_HIP_TRY(hipMalloc(&staging, ref_len));
    hipError_t e = hipMemcpyAsync(staging, ref, ref_len, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      (void)hipFree(staging);
      return set_error(GRIM_EDEVICE, "reference copy failed: %s", hipGetErrorString(e));
    }
    dref = static_cast<const uint8_t*>(staging);
  }
  BuildArgs a{};
  a.ref = dref;
  a.G = ref_len;
  a.B = bin_size;
  a.O = overlap;
  a.q = q;
  a.nb = idx->nb;
  a.tm = idx->tm;
  a.row_words = idx->row_words;
  a.bm = idx->bm;
  a.vec_words = idx->vec_words;
  hipError_t e = hipSuccess;
  {
    ProfSpan ps(PROF_BUILD);
    ps.start(s);
    if (idx->tm) e = launch_build_tm(a, s);
    if (e == hipSuccess && idx->bm) e = launch_build_bm(a, s);
    if (e == hipSuccess && idx->ref) e = launch_ref_codes(dref, ref_len, idx->ref, s);
    ps.stop(s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ps.collect();
  }
  if (staging) (void)hipFree(staging);
  if (e != hipSuccess) return set_error(GRIM_EDEVICE, "index build failed: %s", hipGetErrorString(e));
  *out = idx.release();
  return GRIM_OK;
}

int grim_index_info(const grim_index* idx, grim_index_info_t* out) {
  clear_error();
  if (!idx || !out) return set_error(GRIM_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->ref_len = idx->G;
  out->bin_size = idx->B;
  out->overlap = idx->O;
  out->q = idx->q;
  out->layout = idx->layout;
  out->n_bins = idx->nb;
  out->mask_words = idx->W;
  out->tm_row_words = idx->row_words;
  out->bm_vec_words = idx->vec_words;
  out->device = idx->device;
  out->tm_bytes = idx->tm_bytes;
  out->bm_bytes = idx->bm_bytes;
  out->bits_bytes = idx->nb * (uint64_t)idx->R4 / 8;
  out->ref_bytes = idx->ref_bytes;
  return GRIM_OK;
}

int grim_index_read(const grim_index* idx, uint32_t layout, uint64_t offset, uint64_t nbytes, void* dst) {
  clear_error();
  if (!idx || !dst) return set_error(GRIM_EINVAL, "NULL argument");
  const void* src = nullptr;
  uint64_t size = 0;
  if (layout == GRIM_LAYOUT_TM) { src = idx->tm; size = idx->tm_bytes; }
  else if (layout == GRIM_LAYOUT_BM) { src = idx->bm; size = idx->bm_bytes; }
  else if (layout == GRIM_LAYOUT_REF) { src = idx->ref; size = idx->ref_bytes; }
  else return set_error(GRIM_EINVAL, "layout must be exactly one of GRIM_LAYOUT_TM, GRIM_LAYOUT_BM, GRIM_LAYOUT_REF");
  if (!src) return set_error(GRIM_EINVAL, "layout not present in this index");
  if (offset > size || nbytes > size - offset) return set_error(GRIM_EINVAL, "range outside the layout");
  DeviceGuard dg(idx->device);
  GRIM_HIP_TRY(hipMemcpy(dst, static_cast<const uint8_t*>(src) + offset, nbytes, hipMemcpyDeviceToHost));
  return GRIM_OK;
}

int grim_index_save(const grim_index* idx, const char* path) {
  clear_error();
  if (!idx || !path) return set_error(GRIM_EINVAL, "NULL argument");
  DeviceGuard dg(idx->device);
  std::vector<uint8_t> payload(idx->tm_bytes + idx->bm_bytes + idx->ref_bytes);
  if (idx->tm_bytes) GRIM_HIP_TRY(hipMemcpy(payload.data(), idx->tm, idx->tm_bytes, hipMemcpyDeviceToHost));
  if (idx->bm_bytes)
    GRIM_HIP_TRY(hipMemcpy(payload.data() + idx->tm_bytes, idx->bm, idx->bm_bytes, hipMemcpyDeviceToHost));
  if (idx->ref_bytes)
    GRIM_HIP_TRY(hipMemcpy(payload.data() + idx->tm_bytes + idx->bm_bytes, idx->ref, idx->ref_bytes,
                           hipMemcpyDeviceToHost));
  FileHeader h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = kFileVersion;
  h.header_bytes = sizeof(FileHeader);
  h.G = idx->G;
  h.B = idx->B;
  h.O = idx->O;
  h.q = idx->q;
  h.layout = idx->layout;
  h.nb = idx->nb;
  h.W = idx->W;
  h.row_words = idx->row_words;
  h.vec_words = idx->vec_words;
  h.tm_bytes = idx->tm_bytes;
  h.bm_bytes = idx->bm_bytes;
  h.checksum = fnv1a(0xCBF29CE484222325ull, payload.data(), payload.size());
  std::FILE* f = std::fopen(path, "wb");
  if (!f) return set_error(GRIM_EIO, "cannot open %s for writing", path);
  bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 &&
            (payload.empty() || std::fwrite(payload.data(), payload.size(), 1, f) == 1);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return set_error(GRIM_EIO, "write to %s failed", path);
  return GRIM_OK;
}

int grim_index_load(const char* path, void* hip_stream, grim_index** out) {
  clear_error();
  if (!path || !out) return set_error(GRIM_EINVAL, "NULL argument");
  *out = nullptr;
  std::FILE* f = std::fopen(path, "rb");
  if (!f) return set_error(GRIM_EIO, "cannot open %s", path);
  FileHeader h{};
  if (std::fread(&h, sizeof h, 1, f) != 1) {
    std::fclose(f);
    return set_error(GRIM_EIO, "%s: truncated header", path);
  }
  if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kFileVersion || h.header_bytes != sizeof h) {
    std::fclose(f);
    return set_error(GRIM_EIO, "%s: not a GRIM index file of version %u", path, kFileVersion);
  }
  grim_index probe;
  if (h.B == 0 || h.q < 1 || h.q > 8 || (h.q == 8 && (h.layout & GRIM_LAYOUT_TM)) || h.G < h.q || h.layout == 0 ||
      (h.layout & ~(GRIM_LAYOUT_TM | GRIM_LAYOUT_BM | GRIM_LAYOUT_REF))) {
    std::fclose(f);
    return set_error(GRIM_EIO, "%s: bad parameters in header", path);
  }
  fill_geometry(&probe, h.G, h.B, h.O, h.q, h.layout);
  if (probe.nb != h.nb || probe.W != h.W || probe.row_words != h.row_words || probe.vec_words != h.vec_words ||
      probe.tm_bytes != h.tm_bytes || probe.bm_bytes != h.bm_bytes) {
    std::fclose(f);
    return set_error(GRIM_EIO, "%s: header geometry is inconsistent", path);
  }
  std::vector<uint8_t> payload(h.tm_bytes + h.bm_bytes + probe.ref_bytes);
  const bool ok = payload.empty() || std::fread(payload.data(), payload.size(), 1, f) == 1;
  std::fclose(f);
  if (!ok) return set_error(GRIM_EIO, "%s: truncated payload", path);
  if (fnv1a(0xCBF29CE484222325ull, payload.data(), payload.size()) != h.checksum)
    return set_error(GRIM_EIO, "%s: checksum mismatch", path);
  int dev = 0;
  GRIM_HIP_TRY(hipGetDevice(&dev));
  int rc = check_device(dev);
  if (rc) return rc;
  std::unique_ptr<grim_index, void (*)(grim_index*)> idx(new grim_index, destroy);
  idx->device = dev;
  fill_geometry(idx.get(), h.G, h.B, h.O, h.q, h.layout);
  rc = alloc_layouts(idx.get());
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (idx->tm_bytes) GRIM_HIP_TRY(hipMemcpyAsync(idx->tm, payload.data(), idx->tm_bytes, hipMemcpyHostToDevice, s));
  if (idx->bm_bytes)
    GRIM_HIP_TRY(hipMemcpyAsync(idx->bm, payload.data() + idx->tm_bytes, idx->bm_bytes, hipMemcpyHostToDevice, s));
  if (idx->ref_bytes)
    GRIM_HIP_TRY(hipMemcpyAsync(idx->ref, payload.data() + idx->tm_bytes + idx->bm_bytes, idx->ref_bytes,
                                hipMemcpyHostToDevice, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  *out = idx.release();
  return GRIM_OK;
}

void grim_index_free(grim_index* idx) { grim::destroy(idx); }

int grim_filter_scan(const grim_index* cidx, const grim_reads* rd, uint32_t* mask_out, void* counts_out,
                     uint32_t counts_bytes, void* hip_stream) {
  clear_error();
  int rc = check_reads_args(cidx, rd);
  if (rc) return rc;
  grim_index* idx = const_cast<grim_index*>(cidx);
  if (!(idx->layout & GRIM_LAYOUT_TM)) return set_error(GRIM_EINVAL, "index has no token-major layout");
  if (rd->n_reads && !mask_out) return set_error(GRIM_EINVAL, "mask_out is NULL");
  if (counts_out && counts_bytes != 1 && counts_bytes != 2)
    return set_error(GRIM_EINVAL, "counts_bytes must be 1 or 2");
  if (rd->n_reads == 0) return GRIM_OK;
  std::lock_guard<std::mutex> lk(idx->mu);
  DeviceGuard dg(idx->device);
  apply_cached_config(idx, GRIM_MODE_SCAN, rd->n_reads, rd->n_bases, 0);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ReadView v;
  rc = stage_reads(idx, rd, s, &v);
  if (rc) return rc;
  ProfSpan pt(PROF_TOKENIZE);
  rc = tokenize_reads(idx, rd, v, counts_out && counts_bytes == 1 ? 255u : 65535u, scan_token_shift(idx->q), s,
                      pt);
  if (rc) return rc;
  ScanArgs a{};
  a.tm = idx->tm;
  a.row_words = idx->row_words;
  a.R4 = idx->R4;
  a.q = idx->q;
  a.nb = idx->nb;
  a.W = idx->W;
  a.tokens = idx->ws.tokens;
  a.offsets = v.offsets;
  a.thr = idx->ws.thr;
  a.read_order = nullptr;
  a.n_reads = rd->n_reads;
  a.mask_out = mask_out;
  a.counts_out = counts_out;
  a.counts_bytes = counts_bytes;
  a.status = idx->ws.status;
  const ScanConfig cfg = scan_config_from_env(idx->scan_cfg);
  if (cfg.sort_by_length) {
    rc = grow(&idx->ws.order, &idx->ws.order_cap, rd->n_reads);
    if (rc) return rc;
    if (!idx->ws.hist) GRIM_HIP_TRY(hipMalloc(&idx->ws.hist, length_order_scratch_words() * sizeof(uint32_t)));
    GRIM_HIP_TRY(launch_length_order(v.offsets, rd->n_reads, idx->q, nullptr, idx->ws.hist, idx->ws.order, s));
    a.read_order = idx->ws.order;
  }
  ProfSpan ps(PROF_SCAN);
  ps.start(s);
  GRIM_HIP_TRY(launch_scan_allbins(a, cfg, s));
  ps.stop(s);
  rc = finish_status(idx, s);
  pt.collect();
  ps.collect();
  return rc;
}

int grim_filter_candidates(const grim_index* cidx, const grim_reads* rd, const int64_t* cand_off,
                           const int32_t* cand_bin, uint64_t n_cand, uint16_t* count_out, uint8_t* pass_out,
                           void* hip_stream) {
  clear_error();
  int rc = check_reads_args(cidx, rd);
  if (rc) return rc;
  grim_index* idx = const_cast<grim_index*>(cidx);
  if (!(idx->layout & GRIM_LAYOUT_BM)) return set_error(GRIM_EINVAL, "index has no bin-major layout");
  if (rd->n_reads && !cand_off) return set_error(GRIM_EINVAL, "cand_off is NULL");
  if (n_cand && !cand_bin) return set_error(GRIM_EINVAL, "cand_bin is NULL");
  if (rd->n_reads == 0) return GRIM_OK;
  std::lock_guard<std::mutex> lk(idx->mu);
  DeviceGuard dg(idx->device);
  apply_cached_config(idx, GRIM_MODE_CANDIDATES, rd->n_reads, rd->n_bases, n_cand);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ReadView v;
  rc = stage_reads(idx, rd, s, &v);
  if (rc) return rc;
  ProfSpan pt(PROF_TOKENIZE);
  rc = tokenize_reads(idx, rd, v, 65535u, 0u, s, pt);
  if (rc) return rc;
  CandArgs a{};
  a.bm = idx->bm;
  a.vec_words = idx->vec_words;
  a.R4 = idx->R4;
  a.q = idx->q;
  a.nb = idx->nb;
  a.tokens = idx->ws.tokens;
  a.offsets = v.offsets;
  a.thr = idx->ws.thr;
  a.n_reads = rd->n_reads;
  a.cand_off = cand_off;
  a.cand_bin = cand_bin;
  a.n_cand = n_cand;
  a.count_out = count_out;
  a.pass_out = pass_out;
  a.status = idx->ws.status;
  a.work = idx->ws.status + 4;
  ProfSpan ps(PROF_CAND);
  ps.start(s);
  GRIM_HIP_TRY(launch_scan_candidates(a, cand_config_from_env(idx->cand_cfg), s));
  ps.stop(s);
  rc = finish_status(idx, s);
  pt.collect();
  ps.collect();
  return rc;
}

}  // extern "C"

namespace {

int verify_impl(const grim_index* cidx, const grim_reads* rd, const int64_t* cand_off, const int32_t* cand_bin,
                uint64_t n_cand, const uint8_t* verify_mask, uint16_t* dist_out, uint8_t* match_out,
                void* hip_stream, bool bounded) {
  int rc = check_reads_args(cidx, rd);
  if (rc) return rc;
  grim_index* idx = const_cast<grim_index*>(cidx);
  if (!(idx->layout & GRIM_LAYOUT_REF) || !idx->ref)
    return set_error(GRIM_EINVAL, "index has no reference copy (build it with GRIM_LAYOUT_REF)");
  if (rd->n_reads && !cand_off) return set_error(GRIM_EINVAL, "cand_off is NULL");
  if (n_cand && (!cand_bin || !dist_out || !match_out))
    return set_error(GRIM_EINVAL, "cand_bin, dist_out and match_out must not be NULL");
  if (rd->n_reads == 0 || n_cand == 0) return GRIM_OK;
  std::lock_guard<std::mutex> lk(idx->mu);
  DeviceGuard dg(idx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ReadView v;
  rc = stage_reads(idx, rd, s, &v);
  if (rc) return rc;
  ProfSpan pt(PROF_TOKENIZE);
  rc = tokenize_reads(idx, rd, v, 65535u, 0u, s, pt);  // length checks and thresholds
  if (rc) return rc;
  grim_workspace& ws = idx->ws;
  if (!ws.vbucket) GRIM_HIP_TRY(hipMalloc(&ws.vbucket, kVerifyBuckets * sizeof(uint64_t)));
  if (!ws.vbucket_host)
    GRIM_HIP_TRY(hipHostMalloc(&ws.vbucket_host, 2 * kVerifyBuckets * sizeof(uint64_t), hipHostMallocDefault));
  rc = grow(&ws.vread_sel, &ws.vread_sel_cap, rd->n_reads);
  if (rc) return rc;
  rc = grow(&ws.vchunk_sum, &ws.vchunk_sum_cap, verify_chunks(rd->n_reads) * kVerifyBuckets);
  if (rc) return rc;
  VerifyArgs a{};
  a.ref = idx->ref;
  a.G = idx->G;
  a.B = idx->B;
  a.O = idx->O;
  a.q = idx->q;
  a.nb = idx->nb;
  a.bases = v.bases;
  a.offsets = v.offsets;
  a.thr = ws.thr;
  a.n_reads = rd->n_reads;
  a.cand_off = cand_off;
  a.cand_bin = cand_bin;
  a.n_cand = n_cand;
  a.verify_mask = verify_mask;
  a.dist_out = dist_out;
  a.match_out = match_out;
  a.status = ws.status;
  a.bucket = ws.vbucket;
  a.read_sel = ws.vread_sel;
  a.chunk_sum = ws.vchunk_sum;
  a.bounded = bounded ? 1u : 0u;
  GRIM_HIP_TRY(launch_verify_count(a, s));
  // pairs per length class, and the status of the inputs
  uint64_t* counts = ws.vbucket_host;
  uint64_t* first = ws.vbucket_host + kVerifyBuckets;
  GRIM_HIP_TRY(hipMemcpyAsync(counts, ws.vbucket, kVerifyBuckets * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  rc = finish_status(idx, s);
  pt.collect();
  if (rc) return rc;
  uint64_t total = 0;
  for (uint32_t w = 0; w < kVerifyBuckets; ++w) {
    first[w] = total;
    total += counts[w];
  }
  if (total == 0) return GRIM_OK;
  rc = grow(&ws.vitem_pair, &ws.vitem_cap, total);
  if (rc) return rc;
  rc = grow(&ws.vitem_read, &ws.vitem_read_cap, total);
  if (rc) return rc;
  a.item_pair = ws.vitem_pair;
  a.item_read = ws.vitem_read;
  GRIM_HIP_TRY(launch_verify_scatter(a, s));
  ProfSpan pv(PROF_VERIFY);
  pv.start(s);
  for (uint32_t w = 1; w < kVerifyBuckets; ++w) GRIM_HIP_TRY(launch_verify_align(a, w, first[w], counts[w], s));
  pv.stop(s);
  rc = finish_status(idx, s);
  pv.collect();
  return rc;
}

}  // namespace

extern "C" {

int grim_verify_candidates(const grim_index* cidx, const grim_reads* rd, const int64_t* cand_off,
                           const int32_t* cand_bin, uint64_t n_cand, const uint8_t* verify_mask, uint16_t* dist_out,
                           uint8_t* match_out, void* hip_stream) {
  clear_error();
  return verify_impl(cidx, rd, cand_off, cand_bin, n_cand, verify_mask, dist_out, match_out, hip_stream, false);
}

int grim_verify_candidates_bounded(const grim_index* cidx, const grim_reads* rd, const int64_t* cand_off,
                                   const int32_t* cand_bin, uint64_t n_cand, const uint8_t* verify_mask,
                                   uint16_t* dist_out, uint8_t* match_out, void* hip_stream) {
  clear_error();
  return verify_impl(cidx, rd, cand_off, cand_bin, n_cand, verify_mask, dist_out, match_out, hip_stream, true);
}

}  // extern "C"
