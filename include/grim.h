/*
 * grim.h - C ABI of the GRIM-Filter hot path on AMD Instinct MI355X (gfx950).
 *
 * GRIM-Filter (Kim et al., arXiv 1708.04329) rejects read-mapping locations
 * before alignment. The reference genome is cut into overlapping bins; each
 * bin keeps one existence bit per possible token (q-gram); a read passes a bin
 * when the number of its tokens present there reaches a threshold that no
 * location within E edits can miss.
 *
 * Conventions for every entry point:
 *   - Return value 0 (GRIM_OK) or a negative GRIM_E* code. No exception or
 *     abort crosses this boundary. grim_last_error() gives a message for the
 *     last failure on the calling thread.
 *   - The caller owns every input and output buffer. The library owns
 *     grim_index handles and frees them in grim_index_free.
 *   - "device" buffers are HIP device memory on the device that holds the
 *     index; "host" buffers are ordinary process memory.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on that stream; unless its comment says otherwise
 *     (grim_mask_summary, the batcher and the server), a call returns after
 *     its work on the stream is complete, so outputs are ready on return.
 *   - Bases are ASCII bytes; A, C, G, T are accepted in either case; any
 *     other byte (N, ...) makes every token window that holds it invalid.
 */
#ifndef GRIM_H
#define GRIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRIM_ABI_VERSION 2

enum grim_status {
  GRIM_OK = 0,
  GRIM_EINVAL = -1,     /* an argument or an input value is out of range */
  GRIM_ENOMEM = -2,     /* a device or host allocation failed */
  GRIM_EDEVICE = -3,    /* HIP runtime failure, or no gfx950 device */
  GRIM_EOVERLAP = -4,   /* a read is not covered by the bin overlap: O < L + E - q */
  GRIM_EAGAIN = -5,     /* result not ready yet */
  GRIM_ETIMEDOUT = -6,  /* a wait ran out of time */
  GRIM_ECANCELED = -7,  /* work was cancelled */
  GRIM_EIO = -8         /* index file unreadable, truncated or corrupt */
};

/* Index layouts (bit flags; one index may hold both). */
#define GRIM_LAYOUT_TM 1u /* token-major: row t = bit x of every bin x (all-bins scan) */
#define GRIM_LAYOUT_BM 2u /* bin-major: bin x = its 4^q-bit vector (candidate checks) */
#define GRIM_LAYOUT_REF 4u /* the reference itself, one base code per byte (verification) */

/* grim_reads.flags */
#define GRIM_READS_ALLOW_SHORT_OVERLAP 1u /* compute reads with O < L + E - q instead of
                                             failing with GRIM_EOVERLAP; their result is
                                             still the defined count, but a location within
                                             E edits may then be rejected */

typedef struct grim_index grim_index;

typedef struct {
  uint64_t ref_len;      /* G: reference length in bases */
  uint32_t bin_size;     /* B: bases per bin */
  uint32_t overlap;      /* O: bases each bin extends into the next */
  uint32_t q;            /* token length */
  uint32_t layout;       /* GRIM_LAYOUT_* flags present */
  uint64_t n_bins;       /* ceil(G / B) */
  uint64_t mask_words;   /* W = ceil(n_bins / 32): uint32 words per read in a pass mask */
  uint64_t tm_row_words; /* uint32 words per token-major row (>= W, zero padded) */
  uint32_t bm_vec_words; /* uint32 words per bin-major vector = max(1, 4^q / 32) */
  int32_t device;        /* HIP device ordinal that holds the index */
  uint64_t tm_bytes;     /* device bytes of the token-major layout (0 if absent) */
  uint64_t bm_bytes;     /* device bytes of the bin-major layout (0 if absent) */
  uint64_t bits_bytes;   /* n_bins * 4^q / 8: the existence bits themselves */
  uint64_t ref_bytes;    /* device bytes of the reference copy (GRIM_LAYOUT_REF; 0 if absent) */
} grim_index_info_t;

/* A read set. Read r is bases[offsets[r] .. offsets[r+1]) and has length L_r.
 * Its error budget is E_r = max_edits[r] if max_edits is given, else
 * ceil(err_permille[r] * L_r / 1000) if err_permille is given, else
 * ceil(err_permille_all * L_r / 1000) (paper Section 6, read-existence figure
 * caption: the ceiling of read length times error tolerance). Its threshold
 * is T_r = (L_r - q + 1) - q * E_r (Section 3: an exact match keeps all
 * L - (q - 1) tokens and each error can destroy q of them). */
typedef struct {
  const uint8_t* bases;          /* [n_bases] ASCII bases of all reads, concatenated */
  const int64_t* offsets;        /* [n_reads + 1], non-decreasing, within [0, n_bases] */
  uint64_t n_reads;
  uint64_t n_bases;
  const uint16_t* max_edits;     /* [n_reads] explicit E_r, or NULL */
  const uint16_t* err_permille;  /* [n_reads] per-read error rate in per mille, or NULL */
  uint32_t err_permille_all;     /* error rate for every read when both arrays are NULL */
  uint32_t on_device;            /* 1: bases, offsets, max_edits, err_permille are device
                                    pointers; 0: host pointers (copied in by the call) */
  uint32_t flags;                /* GRIM_READS_* */
  uint32_t reserved;
} grim_reads;

/* ABI version of the loaded library (GRIM_ABI_VERSION it was built with). */
int grim_abi_version(void);

/* Message for the last failed call on this thread ("" if none). The pointer
 * stays valid until the next call on this thread. */
const char* grim_last_error(void);

/* Build the bit vectors of a reference (Section 3, bit vector generation):
 * bin x = [x*B, x*B + B) extended by O bases; bit t of bin x is set when a
 * valid token with code t starts at some s with x*B <= s < x*B + B + O and
 * s <= G - q (a token belongs to the bin holding its first base). Token code:
 * A=0, C=1, G=2, T=3, first base most significant. The bits are stored in the
 * layouts `layout` asks for (GRIM_LAYOUT_TM and/or GRIM_LAYOUT_BM). With
 * GRIM_LAYOUT_REF the index also keeps the reference, one byte per base
 * (0..3 for A, C, G, T in either case, 4 for any other byte), for
 * grim_verify_candidates.
 *   ref, ref_len   reference bases (host, or device if ref_on_device = 1)
 *   bin_size       B >= 1; overlap O >= 0; q in [1, 8] (Section 6.1: a bin's
 *                  vector has 4^q bits; uint16 token codes reach q = 8)
 *   out            receives a new handle, resident on the current HIP device
 * The token-major layout (all-bins scan) takes q <= 7: it stages tiles of
 * 4^q + 1 rows in the 160 KB of LDS of a CU, and at q = 8 even one 32-bin
 * word per row (256 KB) does not fit. Candidate checks (GRIM_LAYOUT_BM, 8 KB
 * vectors) and verification (GRIM_LAYOUT_REF) take q = 8.
 * Errors: GRIM_EINVAL (bad sizes, ref_len < q, more than 2^31 bins,
 *         GRIM_LAYOUT_TM with q = 8), GRIM_ENOMEM, GRIM_EDEVICE. */
int grim_build_index(const uint8_t* ref, uint64_t ref_len, uint32_t ref_on_device,
                     uint32_t bin_size, uint32_t overlap, uint32_t q, uint32_t layout,
                     void* hip_stream, grim_index** out);

/* Describe an index (sizes and layout). */
int grim_index_info(const grim_index* idx, grim_index_info_t* out);

/* Copy `nbytes` of one stored layout, starting at byte `offset`, to host
 * memory `dst` (for inspection and tests). Token-major bytes are row t of
 * tm_row_words uint32 words, bit (x % 32) of word x / 32 = bin x; bin-major
 * bytes are bin x of bm_vec_words words, bit (t % 32) of word t / 32 = token t;
 * reference bytes (GRIM_LAYOUT_REF) are base codes 0..4, one per base.
 * Errors: GRIM_EINVAL (layout absent, range outside it). */
int grim_index_read(const grim_index* idx, uint32_t layout, uint64_t offset, uint64_t nbytes,
                    void* dst);

/* Save the bit vectors for later reuse (Section 3: the bit vectors are built
 * once per reference and saved). The file holds a versioned header with the
 * parameters and a checksum. Errors: GRIM_EIO. */
int grim_index_save(const grim_index* idx, const char* path);

/* Load an index saved by grim_index_save onto the current HIP device.
 * Errors: GRIM_EIO (missing, truncated, bad magic/version/checksum),
 *         GRIM_ENOMEM, GRIM_EDEVICE. */
int grim_index_load(const char* path, void* hip_stream, grim_index** out);

/* Free an index and its device memory (NULL is ignored). */
void grim_index_free(grim_index* idx);

/* All-bins filter (Section 3 steps 1-3 for every bin; Section 4.2: one pass
 * bit per bin per read). For read r and bin x:
 *   count[r][x] = number of token positions i in [0, L_r - q] whose window
 *                 read[i .. i+q) is valid and has its bit set in bin x
 *                 (repeated tokens count every time);
 *   pass[r][x]  = count[r][x] >= T_r.
 * Needs GRIM_LAYOUT_TM.
 *   mask_out    device, [n_reads][mask_words] uint32: bit (x % 32) of word x/32
 *               is pass[r][x]; bits at x >= n_bins are 0.
 *   counts_out  device, NULL or [n_reads][n_bins] counts of counts_bytes each
 *               (1: uint8, every read must have L - q + 1 <= 255; 2: uint16).
 * Errors: GRIM_EINVAL (layout missing, L_r < q, more than 65535 tokens in a
 *         read, bad offsets, counts_bytes), GRIM_EOVERLAP (see
 *         GRIM_READS_ALLOW_SHORT_OVERLAP). On error the outputs are left
 *         unwritten. */
int grim_filter_scan(const grim_index* idx, const grim_reads* reads, uint32_t* mask_out,
                     void* counts_out, uint32_t counts_bytes, void* hip_stream);

/* Candidate-location filter (Section 3 steps 4-5: a location is checked
 * against the bin holding its first base). Read r's candidate bins are
 * cand_bin[cand_off[r] .. cand_off[r+1]); for each entry k the call writes
 *   count_out[k] = count[r][cand_bin[k]] and pass_out[k] = count >= T_r.
 * Needs GRIM_LAYOUT_BM.
 *   cand_off    device, [n_reads + 1] int64, non-decreasing, cand_off[0] = 0
 *   cand_bin    device, [n_cand] int32, each in [0, n_bins)
 *   count_out   device, [n_cand] uint16, or NULL
 *   pass_out    device, [n_cand] uint8 (0/1), or NULL
 * Errors: GRIM_EINVAL (layout missing, bin out of range, bad offsets),
 *         GRIM_EOVERLAP. On error the outputs are unspecified. */
int grim_filter_candidates(const grim_index* idx, const grim_reads* reads,
                           const int64_t* cand_off, const int32_t* cand_bin, uint64_t n_cand,
                           uint16_t* count_out, uint8_t* pass_out, void* hip_stream);

/* grim_filter_candidates without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments, results and errors as
 * grim_filter_candidates, with two differences:
 *   - the reads must be in device memory (on_device = 1);
 *   - the call's scratch (status words, per-read thresholds, token lists) is
 *     a fixed device array of GRIM_STATIC_SCRATCH_BYTES that each GPU the
 *     library runs on holds until the process ends; a call needs
 *     256 + (n_reads + 1) * 4 (rounded up to 256) + 4 * (n_bases + 64 *
 *     n_reads + 128) bytes of it, about 10 MB per 100K reads of 100 bases;
 *     larger calls fail with GRIM_EINVAL (split them, or use
 *     grim_filter_candidates).
 * Every call on one GPU shares that GPU's array. The library runs such calls
 * one at a time per GPU within a process, and a call returns only after its
 * work on hip_stream is complete, so calls cannot overlap; the array keeps
 * the last call's contents, and each call clears what must start at zero.
 * The launch shape is the index's (defaults or grim_tune's choice). */
#define GRIM_STATIC_SCRATCH_BYTES (64ull << 20)
int grim_filter_candidates_static(const grim_index* idx, const grim_reads* reads, const int64_t* cand_off,
                                  const int32_t* cand_bin, uint64_t n_cand, uint16_t* count_out,
                                  uint8_t* pass_out, void* hip_stream);

/* Verification of listed (read, bin) pairs, the step after the filter: a
 * location that passes is aligned with dynamic programming (Section 1,
 * seed-and-extend step 5), and a passing location that yields no mapping
 * counts against the filter (Section 5, evaluation metrics). For entry k,
 * read r and bin x = cand_bin[k]:
 *   dist_out[k]  = the smallest Levenshtein distance (unit-cost substitution,
 *                  insertion, deletion) between the whole read and any
 *                  substring of the bases bin x's tokens cover,
 *                  [x*B, min(x*B + B + O + q - 1, G)); a base other than
 *                  A, C, G, T (either case), in the read or the reference,
 *                  matches nothing; values above 0xFFFE read 0xFFFE;
 *   match_out[k] = dist_out[k] <= E_r (the read's error budget).
 * Entries with verify_mask[k] == 0 are not aligned: dist 0xFFFF, match 0.
 * Pass the filter's pass_out as verify_mask to align only passing pairs, or
 * NULL to align every pair. Needs GRIM_LAYOUT_REF; reads of up to 512
 * bases.
 *   cand_off, cand_bin   as for grim_filter_candidates (device)
 *   verify_mask          device, [n_cand] uint8, or NULL
 *   dist_out, match_out  device, [n_cand] uint16 and uint8
 * Errors: GRIM_EINVAL (no reference in the index, a read longer than 512
 *         bases or shorter than q, bad offsets, bin out of range),
 *         GRIM_ENOMEM. On error the outputs are unspecified. */
int grim_verify_candidates(const grim_index* idx, const grim_reads* reads, const int64_t* cand_off,
                           const int32_t* cand_bin, uint64_t n_cand, const uint8_t* verify_mask,
                           uint16_t* dist_out, uint8_t* match_out, void* hip_stream);

/* ------------------------------------------------------------------------
 * Seeding: the steps before the filter (Section 1, seed-and-extend steps
 * 2-4: seeds of a read are looked up in an index of the reference, giving
 * the candidate locations the filter then checks).
 * ---------------------------------------------------------------------- */
typedef struct grim_seeds grim_seeds; /* opaque; owns device memory */

typedef struct {
  uint64_t ref_len;      /* G */
  uint32_t k;            /* seed length */
  int32_t device;        /* HIP device ordinal holding the table */
  uint64_t n_positions;  /* reference positions whose k bases are all A/C/G/T */
  uint64_t table_bytes;  /* device bytes: (4^k + 1) uint64 starts + uint32 positions */
} grim_seeds_info_t;

/* Seed table of a reference: every position p whose k bases are A, C, G or
 * T (either case), listed under its k-mer (a direct-address table of 4^k
 * buckets).
 *   ref, ref_len   reference bases (host, or device if ref_on_device = 1);
 *                  ref_len < 2^32 (positions are stored as uint32)
 *   k              seed length in [1, 14]
 * Positions within a bucket are in no fixed order; the candidate lists do
 * not depend on it. Any alignment of ref is accepted; a 16-byte aligned
 * device reference (and every host one, which is staged) is read with
 * 16-byte loads. The call returns once the table is built, and ref is not
 * kept.
 * Errors: GRIM_EINVAL, GRIM_ENOMEM, GRIM_EDEVICE. */
int grim_seeds_build(const uint8_t* ref, uint64_t ref_len, uint32_t ref_on_device, uint32_t k, void* hip_stream,
                     grim_seeds** out);
int grim_seeds_info(const grim_seeds* seeds, grim_seeds_info_t* out);
void grim_seeds_free(grim_seeds* seeds);

/* Candidate bins of every read from its seed hits. Seeds are the read's
 * non-overlapping k-mers at offsets 0, k, 2k, ... whose bases are all A, C,
 * G, T; a seed at offset o found at reference position p votes for bin
 * max(p - o, 0) / bin_size. A read's candidates are its bins ranked by votes
 * (more first), then by bin (smaller first), the first `cap` of them, listed
 * by increasing bin: a CSR list in the layout grim_filter_candidates takes.
 *   cand_off    device, [n_reads + 1] int64, written
 *   cand_bin    device, room for n_reads * cap int32; the first *n_cand_out
 *               entries are written
 *   n_cand_out  host, receives the number of candidates
 * Reads may be on the host or the device (grim_reads.on_device); their error
 * budgets are not used. Errors: GRIM_EINVAL (a NULL pointer, bin_size or cap
 * 0, read offsets out of order or outside [0, n_bases]: nothing is written
 * to cand_bin then), GRIM_ENOMEM (the seed hits of one read exceed 2^32),
 * GRIM_EDEVICE. */
int grim_seed_candidates(const grim_seeds* seeds, const grim_reads* reads, uint32_t bin_size, uint32_t cap,
                         int64_t* cand_off, int32_t* cand_bin, uint64_t* n_cand_out, void* hip_stream);

/* grim_verify_candidates with distances bounded by each read's error budget:
 * dist_out[k] is the same smallest edit distance when it is <= E_r and
 * E_r + 1 (at most 0xFFFE) when it is larger; match_out[k] is unchanged
 * (dist <= E_r). A mapper's verification only needs to know whether a
 * location maps within E_r (Section 1, seed-and-extend step 5), and the
 * bound lets each lane advance only the 32-row words of the dynamic program
 * that can still hold a distance <= E_r (Myers 1999, Section 4: the block
 * form with Ukkonen's cutoff), which at most locations is the first one.
 * Arguments, requirements and errors as for grim_verify_candidates. */
int grim_verify_candidates_bounded(const grim_index* idx, const grim_reads* reads, const int64_t* cand_off,
                                   const int32_t* cand_bin, uint64_t n_cand, const uint8_t* verify_mask,
                                   uint16_t* dist_out, uint8_t* match_out, void* hip_stream);

/* Per-read summary of pass masks, for a consumer that keeps the masks in
 * device memory and copies back only a few bytes per read (a read's row is
 * 189 KB at human scale; the masks are the filter's output, Section 3 steps
 * 4-5). For row r of mask, mask_words uint32 words in the layout
 * grim_filter_scan writes (bins past n_bins zero):
 *   pass_count_out[r] = the number of set bits, i.e. of passing bins;
 *   digest_out[r]     = sum over words i of mix64((i << 32) | row[i]), mod 2^64,
 * with mix64 the SplitMix64 output function (Steele, Lea and Flood 2014):
 *   z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
 *   z *= 0x94D049BB133111EB; z ^= z >> 31.
 * Every bit and its position enter the digest, so rows with equal digests are
 * equal with high probability (not certainty).
 *   mask            device, [n_reads][mask_words] uint32, 4-byte aligned
 *   pass_count_out  device, [n_reads] uint32, or NULL
 *   digest_out      device, [n_reads] uint64, or NULL
 * Asynchronous on hip_stream. Errors: GRIM_EINVAL (NULL or misaligned mask,
 * mask_words 0 or >= 2^32), GRIM_EDEVICE. */
int grim_mask_summary(const uint32_t* mask, uint64_t n_reads, uint64_t mask_words, uint32_t* pass_count_out,
                      uint64_t* digest_out, void* hip_stream);

/* Reverse complement of every read (A<->T, C<->G, case kept, other bytes
 * unchanged), read by read with the same offsets: the filter looks at the
 * forward strand only, and a caller covers the other strand by submitting
 * these as more reads. All pointers are device pointers; out has n_bases
 * bytes. Errors: GRIM_EINVAL (a NULL pointer, or offsets out of order or
 * outside [0, n_bases]: such reads are left unwritten, the others are
 * complemented), GRIM_ENOMEM, GRIM_EDEVICE. */
int grim_reverse_complement(const uint8_t* bases, uint64_t n_bases, const int64_t* offsets, uint64_t n_reads,
                            uint8_t* out, void* hip_stream);

/* ------------------------------------------------------------------------
 * Batching layer: launch-shape tuning and a graph-captured steady-state loop.
 * Both drive the same kernels as grim_filter_scan / grim_filter_candidates;
 * the arithmetic (and therefore every output bit) is unchanged.
 * ---------------------------------------------------------------------- */
#define GRIM_MODE_SCAN 1u       /* all-bins filter */
#define GRIM_MODE_CANDIDATES 2u /* candidate-location filter */

/* A launch shape and, after grim_tune, its measured kernel time. */
typedef struct {
  uint32_t mode;               /* GRIM_MODE_* the fields below apply to */
  uint32_t threads;            /* all-bins: threads per workgroup (256, 512, 1024) */
  uint32_t reads_per_chunk;    /* all-bins: most reads per workgroup, i.e. per LDS tile reuse (>= 64); the
                                  launcher deals the reads evenly over a multiple of 8 chunks of at most
                                  this many */
  uint32_t lane_words;         /* all-bins: uint32 words = 32-bin groups per lane (4 or 8) */
  uint32_t cand_waves;         /* candidates: wavefronts per workgroup (0 = by vector size) */
  uint32_t cand_persistent;    /* candidates: 1 = fixed grid with reads handed out by an atomic
                                  counter (uneven reads in one persistent launch); 2 = that grid
                                  for calls of at least 2^20 reads, one wavefront per read below */
  uint32_t cand_groups_per_cu; /* candidates, persistent: workgroups per CU in the fixed grid */
  uint32_t cand_coop;          /* candidates, q >= 5: 1 = 4^q/512 lanes share a pair, each streaming
                                  16-byte chunks of the bin vector; 0 = one lane per pair; 2 (q = 5)
                                  = four reads per wavefront, 16 lanes each, 4 lanes per pair */
  uint32_t n_tried;            /* grim_tune: shapes timed */
  double best_ms;              /* grim_tune: kernel time of the chosen shape on the sample */
  double default_ms;           /* grim_tune: kernel time of the default shape on the sample */
} grim_tune_result;

/* Time every launch shape of one mode on a sample read set and keep the
 * fastest on `idx` for later calls, unless it beats the default shape by less
 * than 5% on the sample (then the default stays; short samples are dominated
 * by launch overhead). The defaults: all-bins 1024 threads, 4096 reads per
 * chunk, 4 words per lane; candidates at q = 5 four reads per wavefront
 * (cand_coop = 2) in workgroups of 2 wavefronts, at q = 6 and 7 cooperative
 * lanes in workgroups of 4 wavefronts, otherwise one lane per pair.
 * The choice is also kept in the file named by the
 * GRIM_TUNE_CACHE environment variable, keyed by mode, q and size class, for
 * later processes). Mode: candidates if cand_off is non-NULL (device arrays
 * as in grim_filter_candidates), else all-bins. The sample should be large
 * enough to fill the GPU. Errors: as the corresponding filter call. */
int grim_tune(grim_index* idx, const grim_reads* sample, const int64_t* cand_off, const int32_t* cand_bin,
              uint64_t n_cand, void* hip_stream, grim_tune_result* out);

/* Read or set the launch shape used by `idx` for one mode (cfg->mode). */
int grim_index_get_config(const grim_index* idx, uint32_t mode, grim_tune_result* out);
int grim_index_set_config(grim_index* idx, const grim_tune_result* cfg);

/* Batcher: a double-buffered, graph-captured loop over batches of reads held
 * in pinned host memory. Each of its two slots owns pinned host buffers,
 * device buffers, a stream and an instantiated hipGraph of the batch's
 * kernels (status reset -> tokenize -> filter), launched between the
 * batch's H2D and D2H copies on the slot's stream. Fill a slot's host
 * buffers, submit, and wait; with two slots, one batch's copies overlap the
 * other's kernels. The launch shape is the index's at
 * creation time (tune first). Results: candidate counts/pass flags land in
 * the slot's pinned host buffers; all-bins masks stay in the slot's device
 * buffer (mask_out), mask_words uint32 per read. */
typedef struct grim_batcher grim_batcher;

#define GRIM_BATCH_EDITS_NONE 0u /* every read uses err_permille_all */
#define GRIM_BATCH_EDITS_MAX 1u  /* `edits` holds E_r per read */
#define GRIM_BATCH_EDITS_ERR 2u  /* `edits` holds e_r per read, per mille */

typedef struct {
  uint8_t* bases;      /* pinned host [max_bases] */
  int64_t* offsets;    /* pinned host [max_reads + 1], offsets[0] = 0 */
  uint16_t* edits;     /* pinned host [max_reads] per edits_kind, or NULL */
  int64_t* cand_off;   /* pinned host [max_reads + 1] (candidates), from 0 to n_cand */
  int32_t* cand_bin;   /* pinned host [max_cand] (candidates) */
  uint16_t* count_out; /* pinned host [max_cand] (candidates): filled when the batch completes */
  uint8_t* pass_out;   /* pinned host [max_cand] (candidates) */
  uint32_t* mask_out;  /* device [max_reads][mask_words] (all-bins) */
} grim_batch_buffers;

/* Create a batcher for `mode` with the given capacities. Errors: GRIM_EINVAL,
 * GRIM_ENOMEM, GRIM_EDEVICE. The index must outlive the batcher. */
int grim_batcher_create(const grim_index* idx, uint32_t mode, uint64_t max_reads, uint64_t max_bases,
                        uint64_t max_cand, uint32_t edits_kind, uint32_t err_permille_all, uint32_t flags,
                        grim_batcher** out);

/* Buffers of slot 0 or 1 (owned by the batcher). */
int grim_batcher_buffers(grim_batcher* b, uint32_t slot, grim_batch_buffers* out);

/* Launch the slot's graph on a batch of n_reads reads / n_bases bases /
 * n_cand pairs already written to its host buffers. Returns at once; the
 * host buffers must not change until grim_batcher_wait. */
int grim_batcher_submit(grim_batcher* b, uint32_t slot, uint64_t n_reads, uint64_t n_bases, uint64_t n_cand);

/* Wait for the slot's batch; returns its status (as the filter calls). */
int grim_batcher_wait(grim_batcher* b, uint32_t slot);

/* The HIP stream of a slot (for ordering device work on its mask_out). */
void* grim_batcher_stream(grim_batcher* b, uint32_t slot);

/* Free a batcher (waits for batches in flight; NULL is ignored). */
void grim_batcher_free(grim_batcher* b);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of all-bins scans against a resident index.
 * Requests (read sets in host memory) are copied at submit, admitted in
 * arrival order while fewer than max_inflight are admitted and their device
 * footprint (inputs, tokens, thresholds, descriptors and their pass masks)
 * fits the free bytes of the server's device arena, a block of HBM taken at
 * creation (by default all free HBM minus reserve_bytes). The continuous
 * policy lets requests that arrive while others run join the next launch:
 * every launch takes up to max_batch_reads reads from the admitted requests,
 * at most slice_reads from each, and launches are spread over n_streams
 * streams. The plain policy runs each request alone as one launch, in arrival
 * order, on one stream (the one-launch-per-batch form, for comparison).
 * A request's pass masks are the same bits grim_filter_scan computes for its
 * reads alone; they stay in device memory until grim_serve_release.
 * ---------------------------------------------------------------------- */
typedef struct grim_server grim_server;

#define GRIM_SERVE_CONTINUOUS 0u
#define GRIM_SERVE_PLAIN 1u

typedef struct {
  uint32_t policy;            /* GRIM_SERVE_CONTINUOUS or GRIM_SERVE_PLAIN */
  uint32_t max_inflight;      /* admitted requests at once (0: 64) */
  uint32_t max_batch_reads;   /* reads per launch, continuous policy (0: 131072) */
  uint32_t slice_reads;       /* reads one request adds to a launch (0: 32768) */
  uint32_t n_streams;         /* device streams for launches (0: 2; plain: 1) */
  uint32_t max_request_reads; /* largest request accepted (0: 65536) */
  uint64_t arena_bytes;       /* device bytes the server serves from (0: free HBM - reserve_bytes) */
  uint64_t reserve_bytes;     /* HBM left free when arena_bytes = 0 */
  uint64_t host_arena_bytes;  /* pinned host bytes for submitted reads (0: 1 GiB) */
  uint32_t flags;             /* GRIM_READS_* for every request */
  uint32_t reserved;
} grim_serve_config;

typedef struct {
  uint64_t ticket;
  int32_t status;        /* GRIM_OK, or the request's error (GRIM_EINVAL, GRIM_EOVERLAP,
                            GRIM_ECANCELED, GRIM_EDEVICE) */
  uint32_t reserved;
  uint64_t n_reads;
  uint64_t mask_words;
  const uint32_t* mask;  /* device [n_reads][mask_words] when status is GRIM_OK; valid until
                            grim_serve_release */
  double latency_ms;     /* submit -> completion observed by the server */
  double queue_ms;       /* submit -> admitted */
} grim_result;

typedef struct {
  uint64_t submitted, completed, failed, rejected, canceled;
  uint64_t reads_completed;
  uint64_t launches;          /* scan launches made */
  uint64_t shared_launches;   /* launches that held reads of two or more requests */
  uint64_t max_requests_per_launch;
  uint64_t peak_device_bytes; /* high-water mark of the arena in use */
  uint64_t arena_bytes;
  double p50_ms, p99_ms, max_ms, mean_ms; /* latency of completed requests (nearest rank) */
  double reads_per_s;         /* completed reads / (last completion - first submit) */
  uint32_t queued, admitted;
} grim_serve_stats_t;

/* Start a server over `idx` (token-major layout) with a scheduler thread.
 * cfg may be NULL for defaults. The index must outlive the server.
 * Errors: GRIM_EINVAL, GRIM_ENOMEM (arena), GRIM_EDEVICE. */
int grim_serve_create(const grim_index* idx, const grim_serve_config* cfg, grim_server** out);

/* Queue a request; its reads (offsets from 0 to n_bases, flags = 0) are
 * copied into the server's pinned staging before the call returns, so the
 * caller may reuse them at once. Host reads (on_device = 0) are copied with
 * memcpy; device reads (on_device = 1, on the index's device) with
 * synchronous device-to-host copies, so their producer must have finished.
 * Errors: GRIM_EINVAL, GRIM_ENOMEM (the request's footprint exceeds the whole
 * arena, so it could never be admitted), GRIM_EAGAIN (host staging full:
 * retry after completions), GRIM_EDEVICE (the server stopped after a device
 * failure, or a copy of device reads failed), GRIM_ECANCELED (shutting down).
 * After a device failure every queued, prepared or waiting request ends with
 * GRIM_EDEVICE; requests whose launches completed keep their results. */
int grim_serve_submit(grim_server* s, const grim_reads* reads, uint64_t* ticket);

/* Result of a request if it has ended (returns its status), else GRIM_EAGAIN. */
int grim_serve_poll(grim_server* s, uint64_t ticket, grim_result* out);

/* Wait up to timeout_ms (< 0: no limit) for a request to end; returns its
 * status, or GRIM_ETIMEDOUT. */
int grim_serve_wait(grim_server* s, uint64_t ticket, int timeout_ms, grim_result* out);

/* Give an ended request's device memory back to the arena and forget it. */
int grim_serve_release(grim_server* s, uint64_t ticket);

/* Cancel a request: queued ones end at once, admitted ones once their
 * launches in flight finish (status GRIM_ECANCELED). */
int grim_serve_cancel(grim_server* s, uint64_t ticket);

/* Counters and latency statistics since creation or the last reset. */
int grim_serve_stats(grim_server* s, grim_serve_stats_t* out);
int grim_serve_reset_stats(grim_server* s);

/* Stop: queued requests are cancelled, admitted ones drain, then all device
 * and host memory of the server is freed (NULL is ignored). */
void grim_serve_destroy(grim_server* s);

/* Kernel timing, recorded with HIP events on the stream each kernel runs on. */
typedef struct {
  uint64_t launches;
  double total_ms;
  double last_ms;
} grim_kernel_time;

typedef struct {
  grim_kernel_time tokenize;    /* read tokenisation + thresholds */
  grim_kernel_time scan;        /* all-bins accumulate + threshold */
  grim_kernel_time candidates;  /* candidate checks */
  grim_kernel_time build;       /* index build */
  grim_kernel_time verify;      /* verification alignments (grim_verify_candidates) */
} grim_profile_t;

/* Turn event timing of library kernels on (1) or off (0). */
int grim_profile_enable(int on);

/* Read the accumulated timings; reset them if `reset` is non-zero. */
int grim_profile_read(grim_profile_t* out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* GRIM_H */
