// grim_filter_candidates_static: the candidate-location filter with no device
// allocation, for callers that cannot allocate (code inside a HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The call computes exactly what grim_filter_candidates computes, with the
// same kernels; only the scratch differs. Instead of the index's workspace
// (which grows with hipMalloc), its status words, per-read thresholds and
// token lists live in `scratch`, a fixed device array of this file. Each GPU
// holds its own copy of the array at its own address, so the host never uses
// the array's name as a device address: the address is taken once per device
// with hipGetSymbolAddress and kept.

#include <cstring>
#include <mutex>

#include "grim_internal.h"

namespace grim {
namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;  // GRIM_STATIC_SCRATCH_BYTES in grim.h
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DeviceScratch {
  uint8_t* ptr = nullptr;  // device address of this device's copy of `scratch`
  std::mutex call_mu;      // one call at a time per device: they share the array
};
DeviceScratch g_scratch[kMaxDevices];
std::mutex g_init_mu;

// Device address of `scratch` on `dev`, which must be the current device.
int scratch_address(int dev, uint8_t** out) {
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (!g_scratch[dev].ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(GRIM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                       hipGetErrorString(e));
    g_scratch[dev].ptr = static_cast<uint8_t*>(p);
  }
  *out = g_scratch[dev].ptr;
  return GRIM_OK;
}

uint64_t up256(uint64_t v) { return (v + 255) / 256 * 256; }

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

}  // namespace
}  // namespace grim

using namespace grim;

extern "C" int grim_filter_candidates_static(const grim_index* cidx, const grim_reads* rd, const int64_t* cand_off,
                                             const int32_t* cand_bin, uint64_t n_cand, uint16_t* count_out,
                                             uint8_t* pass_out, void* hip_stream) {
  clear_error();
  if (!cidx) return set_error(GRIM_EINVAL, "index is NULL");
  if (!rd) return set_error(GRIM_EINVAL, "reads is NULL");
  grim_index* idx = const_cast<grim_index*>(cidx);
  if (!(idx->layout & GRIM_LAYOUT_BM)) return set_error(GRIM_EINVAL, "index has no bin-major layout");
  if (rd->on_device != 1)
    return set_error(GRIM_EINVAL, "reads must be in device memory (on_device = 1): host reads need staging");
  if (rd->flags & ~GRIM_READS_ALLOW_SHORT_OVERLAP) return set_error(GRIM_EINVAL, "unknown reads.flags bits");
  if (rd->n_reads && !rd->offsets) return set_error(GRIM_EINVAL, "reads.offsets is NULL");
  if (rd->n_bases && !rd->bases) return set_error(GRIM_EINVAL, "reads.bases is NULL");
  if (rd->n_reads && !cand_off) return set_error(GRIM_EINVAL, "cand_off is NULL");
  if (n_cand && !cand_bin) return set_error(GRIM_EINVAL, "cand_bin is NULL");
  if (rd->n_reads == 0) return GRIM_OK;
  // scratch layout: status words (status[4] hands out reads to a persistent
  // grid), thresholds, then the token lists (16-byte aligned)
  const uint64_t off_thr = 256;
  const uint64_t off_tok = off_thr + up256((rd->n_reads + 1) * 4);
  if (rd->n_reads > kScratchBytes || rd->n_bases > kScratchBytes ||
      off_tok + token_capacity(rd->n_bases, rd->n_reads) * 4 > kScratchBytes)
    return set_error(GRIM_EINVAL,
                     "%llu reads of %llu bases need %llu scratch bytes, above the fixed %llu "
                     "(GRIM_STATIC_SCRATCH_BYTES); split the call or use grim_filter_candidates",
                     (unsigned long long)rd->n_reads, (unsigned long long)rd->n_bases,
                     (unsigned long long)(off_tok + token_capacity(rd->n_bases, rd->n_reads) * 4),
                     (unsigned long long)kScratchBytes);
  const int dev = idx->device;
  if (dev < 0 || dev >= kMaxDevices) return set_error(GRIM_EDEVICE, "device ordinal %d out of range", dev);
  DeviceGuard dg(dev);
  uint8_t* base = nullptr;
  int rc = scratch_address(dev, &base);
  if (rc) return rc;
  std::lock_guard<std::mutex> call_lk(g_scratch[dev].call_mu);
  CandConfig cfg;
  {
    std::lock_guard<std::mutex> lk(idx->mu);
    cfg = idx->cand_cfg;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  uint32_t* status = reinterpret_cast<uint32_t*>(base);
  int32_t* thr = reinterpret_cast<int32_t*>(base + off_thr);
  uint32_t* tokens = reinterpret_cast<uint32_t*>(base + off_tok);
  // the array keeps the previous call's contents: clear the status words
  GRIM_HIP_TRY(launch_zero_words(status, 8, s));
  TokArgs t{};
  t.bases = rd->bases;
  t.offsets = rd->offsets;
  t.n_reads = rd->n_reads;
  t.n_bases = rd->n_bases;
  t.max_edits = rd->max_edits;
  t.err_pm = rd->err_permille;
  t.err_pm_all = rd->err_permille_all;
  t.q = idx->q;
  t.overlap = idx->O;
  t.flags = rd->flags;
  t.max_tokens = 65535u;
  t.tok_shift = 0;
  t.short_pad = 1;
  t.tokens = tokens;
  t.thr = thr;
  t.status = status;
  GRIM_HIP_TRY(launch_tokenize(t, s));
  CandArgs a{};
  a.bm = idx->bm;
  a.vec_words = idx->vec_words;
  a.R4 = idx->R4;
  a.q = idx->q;
  a.nb = idx->nb;
  a.tokens = tokens;
  a.offsets = rd->offsets;
  a.thr = thr;
  a.n_reads = rd->n_reads;
  a.cand_off = cand_off;
  a.cand_bin = cand_bin;
  a.n_cand = n_cand;
  a.count_out = count_out;
  a.pass_out = pass_out;
  a.status = status;
  a.work = status + 4;
  GRIM_HIP_TRY(launch_scan_candidates(a, cfg, s));
  uint32_t st[8];
  GRIM_HIP_TRY(hipMemcpyAsync(st, status, sizeof st, hipMemcpyDeviceToHost, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  return status_to_error(st[0]);
}
