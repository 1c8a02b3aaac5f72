// Internal declarations shared by the HIP translation units of libgrim.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "grim.h"

namespace grim {

// ---------------------------------------------------------------------------
// Error reporting: every entry point returns a code and leaves a message.
// ---------------------------------------------------------------------------
int set_error(int code, const char* fmt, ...);
const char* last_error();
void clear_error();

#define GRIM_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess)                                                           \
      return ::grim::set_error(_e == hipErrorOutOfMemory ? GRIM_ENOMEM : GRIM_EDEVICE, \
                               "%s failed: %s", #expr, hipGetErrorString(_e));      \
  } while (0)

// Device status words written by kernels (status[0] holds error bits).
enum : uint32_t {
  ST_BAD_LENGTH = 1u,      // L < q or offsets out of order / out of range
  ST_OVERLAP = 2u,         // O < L + E - q without GRIM_READS_ALLOW_SHORT_OVERLAP
  ST_COUNT_U8 = 4u,        // uint8 counts asked for a read with more than 255 tokens
  ST_TOO_LONG = 8u,        // more than 65535 tokens in a read
  ST_BAD_BIN = 16u,        // candidate bin outside [0, n_bins)
  ST_BAD_CAND_OFF = 32u,   // candidate offsets out of order / out of range
  ST_VERIFY_LONG = 64u,    // a read to verify has more than kVerifyMaxLen bases
};
int status_to_error(uint32_t st);

// Loads through a global-memory pointer. A pointer that was itself loaded
// from memory (a request descriptor's token list, say) is a generic pointer
// to the compiler, which then issues flat loads; those also count against the
// LDS wait counter, so every wait for an LDS read would wait for them too.
typedef unsigned int grim_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ldg4(const uint32_t* p) {
  const grim_u32x4 v = *(const __attribute__((address_space(1))) grim_u32x4*)(const void*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t ldg1(const uint32_t* p) {
  return *(const __attribute__((address_space(1))) uint32_t*)(const void*)p;
}

// Token storage: uint32 per token. Read r's tokens start at
// token_base(offsets[r], r) (a multiple of 32 tokens) and are padded with the
// code R4 = 4^q up to the next multiple of 32 above the token count (so at
// least one padding token follows the last real one). Each entry holds
// code << tok_shift: the all-bins scan stores the LDS byte offset of the token's row (shift =
// log2(tile words * 4)), candidate checks store the plain code (shift 0).
// The regions of consecutive reads never overlap, and the buffer needs
// token_capacity(n_bases, n_reads) entries.
__host__ __device__ inline uint64_t token_base(int64_t off, uint64_t r) {
  return ((uint64_t)off + 64ull * r + 31ull) & ~31ull;
}
inline uint64_t token_capacity(uint64_t n_bases, uint64_t n_reads) {
  return n_bases + 64ull * (n_reads + 1) + 64ull;
}

// Tile width in uint32 words of the token-major layout, by q: the tile of
// (4^q + 1) rows must fit the 160 KB of LDS of one CU.
inline int tm_tile_words(uint32_t q) { return q <= 5 ? 32 : (q == 6 ? 8 : 2); }
constexpr uint64_t kTmRowAlign = 64;  // token-major rows padded to 64 words

// ---------------------------------------------------------------------------
// Kernel argument blocks and launchers (one translation unit each).
// ---------------------------------------------------------------------------
// Optional device-resident sizes, so one captured launch serves batches of
// any size up to the capture's maximum: dyn[0] = reads, dyn[1] = bases,
// dyn[2] = candidate pairs.
struct DynSizes {
  uint64_t n_reads, n_bases, n_cand, pad;
};

struct TokArgs {
  const DynSizes* dyn;  // overrides n_reads / n_bases when non-null
  const uint8_t* bases;
  const int64_t* offsets;
  uint64_t n_reads;
  uint64_t n_bases;
  const uint16_t* max_edits;
  const uint16_t* err_pm;
  uint32_t err_pm_all;
  uint32_t q;
  uint32_t overlap;
  uint32_t flags;
  uint32_t max_tokens;  // 255 when uint8 counts are requested, else 65535
  uint32_t tok_shift;   // tokens are stored as code << tok_shift
  uint32_t short_pad;   // 1: a read's entries end at the next multiple of 8 (candidate
                        // checks read no further); 0: past the next multiple of 32 (scans)
  uint32_t pair_order;  // 1: order each read's tokens by the parity of their row (the
                        // all-bins scan with 128-byte tile rows; see launch_tokenize)
  uint32_t* tokens;
  int32_t* thr;
  uint32_t* status;
};
hipError_t launch_tokenize(const TokArgs& a, hipStream_t s);

struct BuildArgs {
  const uint8_t* ref;
  uint64_t G;
  uint32_t B, O, q;
  uint64_t nb;
  uint32_t* tm;          // token-major output or null
  uint64_t row_words;
  uint32_t* bm;          // bin-major output or null
  uint32_t vec_words;
};
hipError_t launch_build_tm(const BuildArgs& a, hipStream_t s);
hipError_t launch_build_bm(const BuildArgs& a, hipStream_t s);
// Reference bytes -> base codes (0..3 for ACGT in either case, 4 otherwise).
hipError_t launch_ref_codes(const uint8_t* ref, uint64_t G, uint8_t* codes, hipStream_t s);

// Verification of (read, bin) pairs: bit-parallel semi-global edit distance
// of the read against the bases of the bin's extent.
constexpr uint32_t kVerifyMaxLen = 512;   // bases per read: 16 words of 32 rows
constexpr uint32_t kVerifyBuckets = 17;   // work lists by words per read, 1..16
constexpr uint32_t kVerifyChunk = 2048;   // reads per workgroup of the list passes
struct VerifyArgs {
  const uint8_t* ref;        // base codes, G bytes
  uint64_t G;
  uint32_t B, O, q;
  uint64_t nb;
  const uint8_t* bases;      // reads, ASCII
  const int64_t* offsets;
  const int32_t* thr;        // T_r (E_r is recovered as (L - q + 1 - T_r) / q)
  uint64_t n_reads;
  const int64_t* cand_off;
  const int32_t* cand_bin;
  uint64_t n_cand;
  const uint8_t* verify_mask;  // or null: every pair
  uint16_t* dist_out;
  uint8_t* match_out;
  uint32_t* status;
  uint64_t* bucket;          // [kVerifyBuckets] pairs to align per class
  uint32_t* read_sel;        // [n_reads] pairs selected per read (first pass)
  uint64_t* chunk_sum;       // [chunks][kVerifyBuckets] pair counts, then first slots
  uint64_t* item_pair;       // work list: pair index
  uint32_t* item_read;       //            and its read
  uint32_t bounded;          // 1: distances above E_r reported as E_r + 1 (Ukkonen's cutoff)
};
// Chunks of reads of the list passes.
uint64_t verify_chunks(uint64_t n_reads);
// Count the pairs to align per class into a.bucket and per chunk (and write
// the outputs of skipped pairs); list positions follow classes in order.
hipError_t launch_verify_count(const VerifyArgs& a, hipStream_t s);
// Fill the work list from the counts and positions of launch_verify_count.
hipError_t launch_verify_scatter(const VerifyArgs& a, hipStream_t s);
// Align work items [first, first + count), all of whose reads have `words`
// 32-base words.
hipError_t launch_verify_align(const VerifyArgs& a, uint32_t words, uint64_t first, uint64_t count,
                               hipStream_t s);

// Per-read descriptor for scans over reads scattered across buffers (served
// requests): token list, output row and threshold of one read.
struct ReadDesc {
  const uint32_t* tok;  // code << scan_token_shift(q), padded to 32 with the zero row
  uint32_t* out;        // mask row: W words
  uint32_t ntok;
  int32_t T;
};

struct ScanArgs {
  const DynSizes* dyn;         // overrides n_reads when non-null
  const ReadDesc* desc;        // per-read descriptors instead of tokens/offsets/thr/mask_out
  const uint32_t* tm;
  uint64_t row_words;
  uint32_t R4;
  uint32_t q;
  uint64_t nb;
  uint64_t W;
  const uint32_t* tokens;      // code << log2(TW * 4): LDS byte offset of the row
  const int64_t* offsets;
  const int32_t* thr;
  const uint32_t* read_order;  // chunk position -> read index, or null for identity
  uint64_t n_reads;
  uint32_t n_tiles;
  uint32_t n_rchunks;          // read chunks (set by the launcher): a multiple of 8
  uint32_t* mask_out;
  void* counts_out;
  uint32_t counts_bytes;
  const uint32_t* status;
};
struct ScanConfig {
  int threads = 1024;         // threads per workgroup (16 waves: 4 per SIMD)
  int reads_per_chunk = 4096; // reads per workgroup (at most)
  int lane_words = 4;         // uint32 words (x32 bins) per lane: 4 or 8
  int sort_by_length = 1;     // process reads longest first (launch_length_order)
};
// Sort reads 0..n-1 by their number of 32-token blocks, longest first, into
// order[]; within a length class, launch position k holds a read whose index
// has the parity of k while both parities last. hist needs
// length_order_scratch_words() words of scratch. Kernels only (graph-safe).
uint64_t length_order_scratch_words();
hipError_t launch_length_order(const int64_t* offsets, uint64_t n, uint32_t q, const DynSizes* dyn, uint32_t* hist,
                               uint32_t* order, hipStream_t s);
// Shift that turns a token code into the LDS byte offset of its tile row.
inline uint32_t scan_token_shift(uint32_t q) {
  const int tw = tm_tile_words(q);
  return tw == 32 ? 7u : (tw == 8 ? 5u : 3u);
}
hipError_t launch_scan_allbins(const ScanArgs& a, const ScanConfig& cfg, hipStream_t s);

struct CandArgs {
  const DynSizes* dyn;         // overrides n_reads / n_cand when non-null
  uint32_t* work;              // persistent mode: work[0] hands out reads to wavefronts
  const uint32_t* bm;
  uint32_t vec_words;
  uint32_t R4;
  uint32_t q;
  uint64_t nb;
  const uint32_t* tokens;      // plain codes (shift 0)
  const int64_t* offsets;
  const int32_t* thr;
  uint64_t n_reads;
  const int64_t* cand_off;
  const int32_t* cand_bin;
  uint64_t n_cand;
  uint16_t* count_out;
  uint8_t* pass_out;
  uint32_t* status;
  uint32_t grab;               // persistent mode: reads taken per counter increment (set at launch)
};
struct CandConfig {
  int waves = 0;         // wavefronts per workgroup (0: by vector size)
  int persistent = 0;    // 1: fixed grid, reads handed out by an atomic counter;
                         // 2: that grid for calls of at least kPersistentMinReads reads, else 0
  int groups_per_cu = 2; // persistent grid size = 256 CUs x groups_per_cu
  int coop = 1;          // 1: VW/16 lanes per pair (q >= 5), 0: one lane per pair,
                         // 2 (q = 5): four reads per wavefront, 16 lanes each
  int planes = 8;        // coop 2: LDS planes per read, 8 (reads above 255 tokens in a
                         // second pass) or 16
};
constexpr uint64_t kPersistentMinReads = 1ull << 20;
// The launch shape an untuned index uses, by vector size: at q = 5 four reads
// per wavefront in workgroups of 2 wavefronts (measured best on the short
// lists of the 100 Mbp workload); at q = 6 and 7 groups of lanes per pair, 4
// wavefronts per workgroup; otherwise one lane per pair.
inline CandConfig default_cand_config(uint32_t vec_words) {
  CandConfig c;
  if (vec_words == 32) {
    c.coop = 2;
    c.waves = 2;
  } else if (vec_words > 32 && vec_words <= 512) {
    c.coop = 1;
    c.waves = 4;
  } else {
    c.coop = 0;
  }
  return c;
}
hipError_t launch_scan_candidates(const CandArgs& a, const CandConfig& cfg, hipStream_t s);
// Zero `n` uint32 words with a kernel (graph-safe, unlike a memset node).
hipError_t launch_zero_words(uint32_t* p, uint32_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Profiling: HIP events around kernels, on the stream they run on.
// ---------------------------------------------------------------------------
enum ProfKind { PROF_TOKENIZE = 0, PROF_SCAN = 1, PROF_CAND = 2, PROF_BUILD = 3, PROF_VERIFY = 4, PROF_N = 5 };
bool profiling();
struct ProfSpan {
  hipEvent_t ev[2] = {nullptr, nullptr};
  ProfKind kind;
  bool on = false;
  explicit ProfSpan(ProfKind k) : kind(k) {}
  ProfSpan(const ProfSpan&) = delete;
  ProfSpan& operator=(const ProfSpan&) = delete;
  void start(hipStream_t s);
  void stop(hipStream_t s);
  void collect();  // after the stream is synchronised
  ~ProfSpan();
};

}  // namespace grim

// ---------------------------------------------------------------------------
// The index handle.
// ---------------------------------------------------------------------------
struct grim_workspace {
  uint32_t* tokens = nullptr;
  uint64_t tokens_cap = 0;
  int32_t* thr = nullptr;
  uint64_t thr_cap = 0;
  uint32_t* status = nullptr;      // device [8]
  uint32_t* status_host = nullptr; // pinned [8]
  uint8_t* staging = nullptr;      // device copies of host-resident inputs
  uint64_t staging_cap = 0;
  uint32_t* order = nullptr;       // scan order (reads sorted by length)
  uint64_t order_cap = 0;
  uint32_t* hist = nullptr;        // 64 words of sort scratch
  uint64_t* vbucket = nullptr;       // device [kVerifyBuckets] verification counts / cursors
  uint64_t* vbucket_host = nullptr;  // pinned [2 * kVerifyBuckets]: counts, first slots
  uint64_t* vitem_pair = nullptr;    // verification work list
  uint32_t* vitem_read = nullptr;
  uint64_t vitem_cap = 0, vitem_read_cap = 0;
  uint32_t* vread_sel = nullptr;     // pairs selected per read
  uint64_t vread_sel_cap = 0;
  uint64_t* vchunk_sum = nullptr;    // per-chunk class counts / first slots
  uint64_t vchunk_sum_cap = 0;
};

struct grim_index {
  grim::ScanConfig scan_cfg;   // launch shape of the all-bins scan (defaults or tuned)
  grim::CandConfig cand_cfg;   // launch shape of candidate checks (defaults or tuned)
  bool scan_tuned = false, cand_tuned = false;
  int device = 0;
  uint64_t G = 0;
  uint32_t B = 0, O = 0, q = 0, layout = 0;
  uint64_t nb = 0, W = 0, row_words = 0;
  uint32_t R4 = 0, vec_words = 0;
  uint32_t* tm = nullptr;
  uint32_t* bm = nullptr;
  uint8_t* ref = nullptr;      // base codes (GRIM_LAYOUT_REF)
  uint64_t tm_bytes = 0, bm_bytes = 0, ref_bytes = 0;
  std::mutex mu;  // guards ws for the duration of a call
  grim_workspace ws;
};
