/*
 * GRIM-Filter CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library or its Python binding may
 * load, link or call this code. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it, to check and to time against.
 *
 * It computes, with plain loops and no blocking or bit tricks, the exact
 * integer result that GRIM-Filter defines (Kim et al., "GRIM-Filter: Fast seed
 * location filtering in DNA read mapping using processing-in-memory
 * technologies", arXiv 1708.04329):
 *
 *   Section 3, bit vector generation: the reference is cut into bins; bin x
 *     has one existence bit per possible token (q-gram), set when a token
 *     whose FIRST base lies in bin x occurs there. Bins overlap so that a read
 *     starting in bin x lies wholly inside it.
 *   Section 6.1: a bit vector holds 4^q bits (4^5 = 1024 for q = 5).
 *   Section 3, steps 1-3: a read's tokens are extracted, their existence bits
 *     in a bin are summed, and the bin passes when the sum meets a threshold.
 *   Section 3, threshold: an exact match yields read_length - (q - 1) tokens;
 *     each error can destroy up to q tokens, so with E errors the threshold is
 *     (L - q + 1) - q*E.
 *   Section 6, caption of the read-existence figure: E is the ceiling of the
 *     read length times the error tolerance e.
 *   Section 3, steps 4-5: a candidate location is checked against the bit of
 *     the bin holding its first base.
 *   Section 1 (seed-and-extend steps 2-4): a mapper selects seeds of a read,
 *     looks them up in an index of the reference, and gets the candidate
 *     locations the filter then checks.
 *   Section 1 (seed-and-extend step 5) and Section 5 (evaluation metrics):
 *     a location that passes the filter is verified by aligning the read to
 *     the reference there with dynamic programming; a passing location that
 *     yields no mapping within the error budget counts against the filter.
 *
 * Conventions the paper leaves open, with the reading taken here (the GPU
 * path implements the same readings independently):
 *   - bins are B bases wide; bin x is extended by O bases into the next bin:
 *     token starts s with x*B <= s < min(x*B + B + O, G - q + 1) count for bin x;
 *     the number of bins is ceil(G / B); the last bin is partial;
 *   - token code: A=0, C=1, G=2, T=3 (case-insensitive), first base most
 *     significant; any other byte makes the window invalid: an invalid
 *     reference window sets no bit, an invalid read window adds 0 but still
 *     counts in L - q + 1;
 *   - every token occurrence of a read counts (repeated tokens add again);
 *   - pass means count >= T; T <= 0 passes every bin;
 *   - E = ceil(e_permille * L / 1000) in integer arithmetic, unless an explicit
 *     per-read E is given;
 *   - verification of (read, bin x) aligns the whole read against any
 *     substring of the bases that bin x's tokens cover, [x*B, min(x*B + B + O
 *     + q - 1, G)), with unit-cost substitutions, insertions and deletions
 *     (Levenshtein distance, free start and end in the reference); a byte
 *     other than A, C, G, T (either case) matches nothing; the location maps
 *     when that distance is at most E;
 *   - seeding: seeds are the read's non-overlapping k-mers at offsets 0, k,
 *     2k, ... whose bases are all A, C, G, T; a seed at offset o found at
 *     reference position p votes for bin max(p - o, 0) / B; a read's
 *     candidates are its bins ranked by votes (more first), then by bin
 *     (smaller first), the first `cap` of them, listed by increasing bin.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Base code of one reference or read byte; -1 for anything but A, C, G, T. */
static int base_code(uint8_t c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

/* Token (q-gram) code of s[0..q): sum of code(s[j]) * 4^(q-1-j); -1 if invalid. */
int64_t oracle_token_code(const uint8_t* s, uint32_t q) {
  int64_t code = 0;
  for (uint32_t j = 0; j < q; ++j) {
    int c = base_code(s[j]);
    if (c < 0) return -1;
    code = code * 4 + c;
  }
  return code;
}

/* Number of possible tokens = length of one bit vector (Section 6.1: 4^q). */
uint64_t oracle_vector_bits(uint32_t q) {
  uint64_t r = 1;
  for (uint32_t j = 0; j < q; ++j) r *= 4;
  return r;
}

/* Number of bins covering a reference of G bases with bins of B bases. */
uint64_t oracle_num_bins(uint64_t G, uint32_t B) {
  if (B == 0) return 0;
  return (G + B - 1) / B;
}

/* Bytes of all bit vectors: one bit per token per bin (Section 6.1 footprint). */
uint64_t oracle_index_bytes(uint64_t n_bins, uint32_t q) {
  return n_bins * oracle_vector_bits(q) / 8;
}

/* Token starts that belong to bin x: [*lo, *hi). */
void oracle_bin_extent(uint64_t x, uint64_t G, uint32_t B, uint32_t O, uint32_t q,
                       uint64_t* lo, uint64_t* hi) {
  uint64_t last_start_plus_one = (G >= q) ? G - q + 1 : 0;
  uint64_t a = x * (uint64_t)B;
  uint64_t b = a + (uint64_t)B + (uint64_t)O;
  if (b > last_start_plus_one) b = last_start_plus_one;
  if (a > b) a = b;
  *lo = a;
  *hi = b;
}

/* Bit vectors, one byte per existence bit: bits[x * 4^q + t] is 1 when token t
 * starts inside bin x's extent (Section 3, bit vector generation). */
int oracle_build_bits(const uint8_t* ref, uint64_t G, uint32_t B, uint32_t O, uint32_t q,
                      uint8_t* bits, int nthreads) {
  if (B == 0 || q == 0 || q > 12) return -1;
  const uint64_t nb = oracle_num_bins(G, B);
  const uint64_t R = oracle_vector_bits(q);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t x = 0; x < (int64_t)nb; ++x) {
    uint8_t* v = bits + (uint64_t)x * R;
    memset(v, 0, R);
    uint64_t lo, hi;
    oracle_bin_extent((uint64_t)x, G, B, O, q, &lo, &hi);
    for (uint64_t s = lo; s < hi; ++s) {
      int64_t t = oracle_token_code(ref + s, q);
      if (t >= 0) v[t] = 1;
    }
  }
  return 0;
}

/* E from an error rate in per mille: ceil(e * L / 1000) (Section 6, caption of
 * the read-existence figure). */
uint32_t oracle_max_edits(uint32_t L, uint32_t e_permille) {
  return (uint32_t)(((uint64_t)L * e_permille + 999) / 1000);
}

/* Threshold (Section 3): tokens of an exact match minus q per error. */
int64_t oracle_threshold(uint32_t L, uint32_t q, uint32_t E) {
  return ((int64_t)L - (int64_t)q + 1) - (int64_t)q * (int64_t)E;
}

/* Sum of the existence bits of every token of one read in one bin (steps 1-2). */
uint32_t oracle_count(const uint8_t* bits_of_bin, const uint8_t* read, uint32_t L, uint32_t q) {
  uint32_t count = 0;
  for (uint32_t i = 0; i + q <= L; ++i) {
    int64_t t = oracle_token_code(read + i, q);
    if (t >= 0 && bits_of_bin[t]) count += 1;
  }
  return count;
}

/* Error budget E_r of read r: the explicit per-read value if given, else the
 * ceiling rule on the read's own rate, else on the rate shared by all reads. */
static uint32_t read_budget(const int64_t* offsets, uint64_t r, const uint16_t* max_edits,
                            const uint16_t* err_pm_per_read, uint32_t err_permille) {
  uint32_t L = (uint32_t)(offsets[r + 1] - offsets[r]);
  if (max_edits) return max_edits[r];
  if (err_pm_per_read) return oracle_max_edits(L, err_pm_per_read[r]);
  return oracle_max_edits(L, err_permille);
}

static int64_t read_threshold(const int64_t* offsets, uint64_t r, uint32_t q,
                              const uint16_t* max_edits, const uint16_t* err_pm_per_read,
                              uint32_t err_permille) {
  uint32_t L = (uint32_t)(offsets[r + 1] - offsets[r]);
  return oracle_threshold(L, q, read_budget(offsets, r, max_edits, err_pm_per_read, err_permille));
}

/* Threshold of every read, for checking the GPU's per-read threshold table. */
void oracle_thresholds(const int64_t* offsets, uint64_t n, uint32_t q, const uint16_t* max_edits,
                       const uint16_t* err_pm_per_read, uint32_t err_permille, int64_t* T_out) {
  for (uint64_t r = 0; r < n; ++r)
    T_out[r] = read_threshold(offsets, r, q, max_edits, err_pm_per_read, err_permille);
}

/* All-bins filter (Section 3 steps 1-3 for every bin): counts[r * nb + x] and
 * pass[r * nb + x] = (count >= T_r). Either output may be NULL. */
int oracle_scan_all(const uint8_t* bits, uint64_t nb, uint32_t q, const uint8_t* bases,
                    const int64_t* offsets, uint64_t n, const uint16_t* max_edits,
                    const uint16_t* err_pm_per_read, uint32_t err_permille,
                    uint16_t* counts, uint8_t* pass, int nthreads) {
  const uint64_t R = oracle_vector_bits(q);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const int64_t cells = (int64_t)(n * nb);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t c = 0; c < cells; ++c) {
    uint64_t r = (uint64_t)c / nb, x = (uint64_t)c % nb;
    uint32_t L = (uint32_t)(offsets[r + 1] - offsets[r]);
    uint32_t cnt = oracle_count(bits + x * R, bases + offsets[r], L, q);
    int64_t T = read_threshold(offsets, r, q, max_edits, err_pm_per_read, err_permille);
    if (counts) counts[c] = (uint16_t)cnt;
    if (pass) pass[c] = (int64_t)cnt >= T ? 1 : 0;
  }
  return 0;
}

/* Candidate mode (Section 3 steps 4-5): read r's candidate bins are
 * cand_bin[cand_off[r] .. cand_off[r+1]); outputs are in the same order. */
int oracle_scan_candidates(const uint8_t* bits, uint64_t nb, uint32_t q, const uint8_t* bases,
                           const int64_t* offsets, uint64_t n, const uint16_t* max_edits,
                           const uint16_t* err_pm_per_read, uint32_t err_permille,
                           const int64_t* cand_off, const int32_t* cand_bin,
                           uint16_t* counts, uint8_t* pass, int nthreads) {
  const uint64_t R = oracle_vector_bits(q);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
  for (int64_t r = 0; r < (int64_t)n; ++r) {
    uint32_t L = (uint32_t)(offsets[r + 1] - offsets[r]);
    int64_t T = read_threshold(offsets, (uint64_t)r, q, max_edits, err_pm_per_read, err_permille);
    for (int64_t k = cand_off[r]; k < cand_off[r + 1]; ++k) {
      int32_t x = cand_bin[k];
      if (x < 0 || (uint64_t)x >= nb) { bad = 1; continue; }
      uint32_t cnt = oracle_count(bits + (uint64_t)x * R, bases + offsets[r], L, q);
      if (counts) counts[k] = (uint16_t)cnt;
      if (pass) pass[k] = (int64_t)cnt >= T ? 1 : 0;
    }
  }
  return bad ? -1 : 0;
}

/* Smallest edit distance between the whole read and any substring of text:
 * the textbook dynamic program over one column at a time. Row i of a column
 * holds the distance of read[0..i) to the best substring ending at that text
 * position; row 0 is 0 in every column (the substring may start anywhere). */
uint32_t oracle_semiglobal_distance(const uint8_t* read, uint32_t L, const uint8_t* text, uint64_t n) {
  uint32_t* col = (uint32_t*)malloc(sizeof(uint32_t) * (L + 1));
  if (!col) return UINT32_MAX;
  for (uint32_t i = 0; i <= L; ++i) col[i] = i;  /* empty text prefix */
  uint32_t best = col[L];
  for (uint64_t j = 0; j < n; ++j) {
    const int tc = base_code(text[j]);
    uint32_t diag = col[0];  /* previous column, row i - 1 */
    col[0] = 0;
    for (uint32_t i = 1; i <= L; ++i) {
      const int rc = base_code(read[i - 1]);
      const uint32_t sub = diag + ((rc >= 0 && rc == tc) ? 0u : 1u);
      const uint32_t del = col[i] + 1;       /* text base skipped */
      const uint32_t ins = col[i - 1] + 1;   /* read base skipped */
      uint32_t v = sub < del ? sub : del;
      if (ins < v) v = ins;
      diag = col[i];
      col[i] = v;
    }
    if (col[L] < best) best = col[L];
  }
  free(col);
  return best;
}

/* Bases that bin x's tokens cover: [*lo, *hi). */
void oracle_bin_bases(uint64_t x, uint64_t G, uint32_t B, uint32_t O, uint32_t q, uint64_t* lo, uint64_t* hi) {
  uint64_t a, b;
  oracle_bin_extent(x, G, B, O, q, &a, &b);
  *lo = a;
  *hi = b > a ? b + q - 1 : a;
}

/* Verification of listed (read, bin) pairs: dist[k] = semi-global distance of
 * read r against bin cand_bin[k]'s bases and match[k] = (dist <= E_r). Pairs
 * with verify_mask[k] == 0 (when a mask is given) are skipped: dist 0xFFFF,
 * match 0. Distances above 0xFFFE are reported as 0xFFFE. */
int oracle_verify(const uint8_t* ref, uint64_t G, uint32_t B, uint32_t O, uint32_t q, const uint8_t* bases,
                  const int64_t* offsets, uint64_t n, const uint16_t* max_edits, const uint16_t* err_pm_per_read,
                  uint32_t err_permille, const int64_t* cand_off, const int32_t* cand_bin,
                  const uint8_t* verify_mask, uint16_t* dist, uint8_t* match, int nthreads) {
  const uint64_t nb = oracle_num_bins(G, B);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int64_t r = 0; r < (int64_t)n; ++r) {
    const uint32_t L = (uint32_t)(offsets[r + 1] - offsets[r]);
    const uint32_t E = read_budget(offsets, (uint64_t)r, max_edits, err_pm_per_read, err_permille);
    for (int64_t k = cand_off[r]; k < cand_off[r + 1]; ++k) {
      const int32_t x = cand_bin[k];
      if (x < 0 || (uint64_t)x >= nb) { bad = 1; continue; }
      if (verify_mask && !verify_mask[k]) {
        dist[k] = 0xFFFF;
        match[k] = 0;
        continue;
      }
      uint64_t lo, hi;
      oracle_bin_bases((uint64_t)x, G, B, O, q, &lo, &hi);
      const uint32_t d = oracle_semiglobal_distance(bases + offsets[r], L, ref + lo, hi - lo);
      dist[k] = (uint16_t)(d > 0xFFFE ? 0xFFFE : d);
      match[k] = d <= E ? 1 : 0;
    }
  }
  return bad ? -1 : 0;
}

/* Bounded verification: as oracle_verify, but an aligned pair whose distance
 * exceeds the read's budget E_r reads E_r + 1 (at most 0xFFFE). A mapper's
 * verification only has to decide whether the location maps within E_r
 * (Section 1, seed-and-extend step 5), so distances past the budget carry no
 * more information than "over". Skipped pairs keep 0xFFFF; match flags are
 * oracle_verify's. */
int oracle_verify_bounded(const uint8_t* ref, uint64_t G, uint32_t B, uint32_t O, uint32_t q,
                          const uint8_t* bases, const int64_t* offsets, uint64_t n, const uint16_t* max_edits,
                          const uint16_t* err_pm_per_read, uint32_t err_permille, const int64_t* cand_off,
                          const int32_t* cand_bin, const uint8_t* verify_mask, uint16_t* dist, uint8_t* match,
                          int nthreads) {
  int rc = oracle_verify(ref, G, B, O, q, bases, offsets, n, max_edits, err_pm_per_read, err_permille, cand_off,
                         cand_bin, verify_mask, dist, match, nthreads);
  if (rc != 0) return rc;
  for (uint64_t r = 0; r < n; ++r) {
    const uint32_t E = read_budget(offsets, r, max_edits, err_pm_per_read, err_permille);
    for (int64_t k = cand_off[r]; k < cand_off[r + 1]; ++k) {
      if (dist[k] == 0xFFFF) continue; /* not aligned */
      if (dist[k] > E) dist[k] = (uint16_t)(E + 1 < 0xFFFE ? E + 1 : 0xFFFE);
    }
  }
  return 0;
}

/* One reference k-mer occurrence: code and start position. */
typedef struct {
  uint64_t code;
  uint64_t pos;
} kmer_pos;

static int cmp_kmer_pos(const void* a, const void* b) {
  const kmer_pos* x = (const kmer_pos*)a;
  const kmer_pos* y = (const kmer_pos*)b;
  if (x->code != y->code) return x->code < y->code ? -1 : 1;
  if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
  return 0;
}

typedef struct {
  int64_t bin;
  uint64_t votes;
} bin_votes;

static int cmp_int64(const void* a, const void* b) {
  const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* more votes first, then the smaller bin */
static int cmp_rank(const void* a, const void* b) {
  const bin_votes* x = (const bin_votes*)a;
  const bin_votes* y = (const bin_votes*)b;
  if (x->votes != y->votes) return x->votes > y->votes ? -1 : 1;
  return x->bin < y->bin ? -1 : (x->bin > y->bin ? 1 : 0);
}

static int cmp_bin(const void* a, const void* b) {
  const bin_votes* x = (const bin_votes*)a;
  const bin_votes* y = (const bin_votes*)b;
  return x->bin < y->bin ? -1 : (x->bin > y->bin ? 1 : 0);
}

/* Seed-hit candidate bins of every read (the seeding steps that precede the
 * filter). cand_off[n + 1] and cand_bin (room for n * cap entries) receive a
 * CSR list; returns the number of candidates, or -1 on bad arguments. The
 * reference's k-mers are listed and sorted by code, and each seed's hits are
 * the run of its code in that list. */
int64_t oracle_seed_candidates(const uint8_t* ref, uint64_t G, const uint8_t* bases, const int64_t* offsets,
                               uint64_t n, uint32_t k, uint32_t B, uint32_t cap, int64_t* cand_off,
                               int32_t* cand_bin) {
  if (k == 0 || k > 16 || B == 0) return -1;
  uint64_t m = 0;
  kmer_pos* table = (kmer_pos*)malloc(sizeof(kmer_pos) * (G >= k ? G - k + 1 : 1));
  if (!table) return -1;
  for (uint64_t p = 0; p + k <= G; ++p) {
    int64_t code = oracle_token_code(ref + p, k);
    if (code < 0) continue;
    table[m].code = (uint64_t)code;
    table[m].pos = p;
    ++m;
  }
  qsort(table, m, sizeof(kmer_pos), cmp_kmer_pos);
  int64_t total = 0;
  for (uint64_t r = 0; r < n; ++r) {
    const uint8_t* rd = bases + offsets[r];
    const int64_t L = offsets[r + 1] - offsets[r];
    /* every hit's bin, with repeats */
    uint64_t nh = 0, cap_h = 64;
    int64_t* hits = (int64_t*)malloc(sizeof(int64_t) * cap_h);
    for (int64_t o = 0; o + (int64_t)k <= L; o += k) {
      int64_t code = oracle_token_code(rd + o, k);
      if (code < 0) continue;
      /* first entry with this code (binary search), then its run */
      uint64_t lo = 0, hi = m;
      while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (table[mid].code < (uint64_t)code) lo = mid + 1;
        else hi = mid;
      }
      for (uint64_t h = lo; h < m && table[h].code == (uint64_t)code; ++h) {
        int64_t loc = (int64_t)table[h].pos - o;
        if (loc < 0) loc = 0;
        if (nh == cap_h) {
          cap_h *= 2;
          hits = (int64_t*)realloc(hits, sizeof(int64_t) * cap_h);
        }
        hits[nh++] = loc / (int64_t)B;
      }
    }
    /* votes per bin */
    qsort(hits, nh, sizeof(int64_t), cmp_int64);
    bin_votes* bv = (bin_votes*)malloc(sizeof(bin_votes) * (nh ? nh : 1));
    uint64_t nb_r = 0;
    for (uint64_t i = 0; i < nh;) {
      uint64_t j = i;
      while (j < nh && hits[j] == hits[i]) ++j;
      bv[nb_r].bin = hits[i];
      bv[nb_r].votes = j - i;
      ++nb_r;
      i = j;
    }
    if (nb_r > cap) {
      qsort(bv, nb_r, sizeof(bin_votes), cmp_rank);
      nb_r = cap;
      qsort(bv, nb_r, sizeof(bin_votes), cmp_bin);
    }
    cand_off[r] = total;
    for (uint64_t i = 0; i < nb_r; ++i) cand_bin[total + (int64_t)i] = (int32_t)bv[i].bin;
    total += (int64_t)nb_r;
    free(bv);
    free(hits);
  }
  cand_off[n] = total;
  free(table);
  return total;
}

/* Threads the parallel loops will use. */
int oracle_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
}
