// Seeded synthetic inputs for the GRIM-Filter hot path: genomes, reads with a
// known edit script, and seed-hit candidate lists.
//
// This module is shared by the CPU oracle and the GPU path and therefore holds
// none of the filter's arithmetic (no bins, no q-gram presence bits, no
// thresholds). Candidate generation uses exact k-mer seed hits, which is the
// read mapper's step that runs before the filter (paper Section 1, seed-and-
// extend flow), not the filter itself.
//
// Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15,
// then two xor-shift-multiply rounds and a final xor-shift. Every read (and
// every genome block) draws from its own stream, so generation is
// deterministic whatever the thread count.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next() { s += kGolden; return mix64(s); }
  // uniform double in [0, 1) from the top 53 bits
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  // uniform integer in [0, n) by 128-bit multiply (Lemire); n > 0
  uint64_t below(uint64_t n) {
    return (uint64_t)(((unsigned __int128)next() * (unsigned __int128)n) >> 64);
  }
};

// Independent stream for item `idx` under `seed`.
inline uint64_t stream_seed(uint64_t seed, uint64_t tag, uint64_t idx) {
  return mix64(seed ^ mix64(tag * kGolden + 0x632BE59BD9B4E019ull) ^ mix64(idx + 0x1234567ull));
}

const uint8_t kBases[4] = {'A', 'C', 'G', 'T'};

inline int code_of(uint8_t c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

}  // namespace

extern "C" {

typedef struct {
  uint64_t seed;
  uint64_t length;
  double repeat_frac;     // stop placing copies once placed bases >= repeat_frac * length
  uint32_t n_families;    // number of repeat families (consensus sequences)
  uint32_t fam_len_lo;    // consensus length range
  uint32_t fam_len_hi;
  uint32_t fam_len_mode;  // 0: uniform in [lo, hi]; 1: half the families lo, half hi,
                          //    copies alternate so each class gets ~half the repeat bases
  double div_lo;          // per-copy divergence, uniform in [div_lo, div_hi]
  double div_hi;
  double indel_share;     // share of divergence events that are indels (rest substitutions)
} synth_genome_params;

// Uniform i.i.d. ACGT background, then interspersed repeat copies written over it.
// Returns the number of repeat bases placed (counting overlaps twice), or -1.
int64_t synth_genome(const synth_genome_params* p, uint8_t* out) {
  if (!p || !out) return -1;
  const uint64_t G = p->length;
  // Background: block b of 32 bases takes 2 bits each from one 64-bit draw.
  const uint64_t nblk = (G + 31) / 32;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < (int64_t)nblk; ++b) {
    uint64_t r = mix64(p->seed * kGolden + mix64((uint64_t)b + 0x51ED2701ull));
    uint64_t base = (uint64_t)b * 32;
    uint64_t end = std::min<uint64_t>(base + 32, G);
    for (uint64_t i = base; i < end; ++i) { out[i] = kBases[r & 3]; r >>= 2; }
  }
  if (p->repeat_frac <= 0.0 || p->n_families == 0) return 0;

  SplitMix64 rng(stream_seed(p->seed, 1, 0));
  std::vector<std::vector<uint8_t>> fam(p->n_families);
  for (uint32_t f = 0; f < p->n_families; ++f) {
    uint32_t len;
    if (p->fam_len_mode == 1) len = (f & 1) ? p->fam_len_hi : p->fam_len_lo;
    else len = p->fam_len_lo + (uint32_t)rng.below((uint64_t)(p->fam_len_hi - p->fam_len_lo) + 1);
    fam[f].resize(len);
    for (uint32_t i = 0; i < len; ++i) fam[f][i] = kBases[rng.next() & 3];
  }
  const double target = p->repeat_frac * (double)G;
  double placed = 0.0, placed_short = 0.0, placed_long = 0.0;
  std::vector<uint8_t> copy;
  uint64_t attempts = 0;
  while (placed < target && ++attempts < (1ull << 40)) {
    uint32_t f;
    if (p->fam_len_mode == 1) {
      // pick the class that is behind in placed bases, then a family of that class
      uint32_t cls = placed_short <= placed_long ? 0u : 1u;
      uint32_t nclass = (p->n_families + 1 - cls) / 2;
      if (nclass == 0) cls ^= 1u, nclass = (p->n_families + 1 - cls) / 2;
      f = cls + 2 * (uint32_t)rng.below(nclass);
    } else {
      f = (uint32_t)rng.below(p->n_families);
    }
    const std::vector<uint8_t>& cons = fam[f];
    double d = p->div_lo + (p->div_hi - p->div_lo) * rng.uniform();
    copy.clear();
    for (size_t i = 0; i < cons.size(); ++i) {
      if (rng.uniform() < d) {
        double u = rng.uniform();
        if (u < p->indel_share * 0.5) {          // insertion before this base
          copy.push_back(kBases[rng.next() & 3]);
          copy.push_back(cons[i]);
        } else if (u < p->indel_share) {         // deletion of this base
        } else {                                 // substitution by a different base
          int c = code_of(cons[i]);
          copy.push_back(kBases[(c + 1 + (int)rng.below(3)) & 3]);
        }
      } else {
        copy.push_back(cons[i]);
      }
    }
    if (copy.empty() || copy.size() >= G) {
      if (cons.size() >= G) return -2;  // a family longer than the genome can never be placed
      continue;
    }
    uint64_t pos = rng.below(G - copy.size() + 1);
    std::memcpy(out + pos, copy.data(), copy.size());
    placed += (double)copy.size();
    if (p->fam_len_mode == 1) ((f & 1) ? placed_long : placed_short) += (double)copy.size();
  }
  return (int64_t)placed;
}

typedef struct {
  uint64_t seed;
  uint64_t n_reads;
  uint32_t n_len;        // read-length mix: lens[i] with weight len_w[i]
  uint32_t lens[4];
  uint32_t len_w[4];
  uint32_t n_err;        // error-rate mix in per mille: err_pm[i] with weight err_w[i]
  uint32_t err_pm[8];
  uint32_t err_w[8];
  uint32_t edit_mode;    // 0: `edits` edits, types drawn by w_sub:w_ins:w_del
                         // 1: floor(err_pm * L / 1000) edits, types by the weights
                         // 2: n_sub substitutions plus n_indel indels (ins:del 1:1)
  uint32_t edits;
  uint32_t w_sub, w_ins, w_del;
  uint32_t n_sub, n_indel;
} synth_read_params;

static uint32_t pick_weighted(SplitMix64& rng, uint32_t n, const uint32_t* w) {
  uint64_t tot = 0;
  for (uint32_t i = 0; i < n; ++i) tot += w[i];
  if (tot == 0) return 0;
  uint64_t u = rng.below(tot);
  for (uint32_t i = 0; i < n; ++i) { if (u < w[i]) return i; u -= w[i]; }
  return n - 1;
}

// Read lengths only (pass 1), so the caller can size the base buffer.
int synth_read_lengths(const synth_read_params* p, uint32_t* len_out) {
  if (!p || !len_out || p->n_len == 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < (int64_t)p->n_reads; ++r) {
    SplitMix64 rng(stream_seed(p->seed, 2, (uint64_t)r));
    len_out[r] = p->lens[pick_weighted(rng, p->n_len, p->len_w)];
  }
  return 0;
}

// Reads sampled at uniform reference positions with an exact edit script.
// offsets[n+1] must already hold the prefix sums of synth_read_lengths.
// Outputs per read: truth start, reference span consumed, error rate (per mille),
// number of edits applied.
int synth_reads(const synth_read_params* p, const uint8_t* genome, uint64_t G,
                const int64_t* offsets, uint8_t* bases, uint64_t* truth_pos,
                uint32_t* span_out, uint16_t* err_pm_out, uint16_t* n_edits_out) {
  if (!p || !genome || !offsets || !bases) return -1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
  for (int64_t r = 0; r < (int64_t)p->n_reads; ++r) {
    SplitMix64 rng(stream_seed(p->seed, 2, (uint64_t)r));
    const uint32_t L = p->lens[pick_weighted(rng, p->n_len, p->len_w)];
    if ((int64_t)L != offsets[r + 1] - offsets[r]) { bad |= 1; continue; }
    SplitMix64 er(stream_seed(p->seed, 3, (uint64_t)r));
    const uint32_t epm = p->n_err ? p->err_pm[pick_weighted(er, p->n_err, p->err_w)] : 0;
    // edit script over read positions: type per position (0 none, 1 S, 2 I, 3 D)
    std::vector<uint8_t> type(L, 0);
    uint32_t k;
    if (p->edit_mode == 0) k = p->edits;
    else if (p->edit_mode == 1) k = (uint32_t)(((uint64_t)epm * L) / 1000);
    else k = p->n_sub + p->n_indel;
    if (k > L) k = L;
    // k distinct read positions by partial Fisher-Yates
    std::vector<uint32_t> perm(L);
    for (uint32_t i = 0; i < L; ++i) perm[i] = i;
    for (uint32_t i = 0; i < k; ++i) {
      uint32_t j = i + (uint32_t)er.below(L - i);
      std::swap(perm[i], perm[j]);
      uint8_t t;
      if (p->edit_mode == 2) t = i < p->n_sub ? 1 : (er.below(2) ? 2 : 3);
      else { const uint32_t w[3] = {p->w_sub, p->w_ins, p->w_del}; t = (uint8_t)(1 + pick_weighted(er, 3, w)); }
      type[perm[i]] = t;
    }
    uint32_t ndel = 0, nins = 0;
    for (uint32_t i = 0; i < L; ++i) { ndel += type[i] == 3; nins += type[i] == 2; }
    const uint64_t span_max = (uint64_t)L + ndel;  // reference bases consumed at most
    if (span_max > G) { bad |= 2; continue; }
    const uint64_t start = er.below(G - span_max + 1);
    uint8_t* out = bases + offsets[r];
    uint64_t j = start;
    for (uint32_t i = 0; i < L; ++i) {
      switch (type[i]) {
        case 0: out[i] = genome[j++]; break;
        case 1: {
          int c = code_of(genome[j++]);
          if (c < 0) c = 0;
          out[i] = kBases[(c + 1 + (int)er.below(3)) & 3];
          break;
        }
        case 2: out[i] = kBases[er.next() & 3]; break;       // inserted read base
        case 3: ++j; out[i] = genome[j++]; break;            // reference base skipped
      }
    }
    if (truth_pos) truth_pos[r] = start;
    if (span_out) span_out[r] = (uint32_t)(j - start);
    if (err_pm_out) err_pm_out[r] = (uint16_t)epm;
    if (n_edits_out) n_edits_out[r] = (uint16_t)k;
    (void)nins;
  }
  return bad ? -2 : 0;
}

// Exact k-mer seed hits (k <= 14): non-overlapping seeds at read offsets
// 0, k, 2k, ... (while offset + k <= L). Each hit h of the seed at offset o
// proposes location max(h - o, 0) and bin location / bin_size. Bins are
// deduplicated with one vote per hit, ranked by votes (descending) then bin
// (ascending), capped at `cap`, and stored in ascending bin order.
// cand_off[n+1] receives the CSR offsets; cand_bin needs n * cap entries.
// Returns the total number of candidates, or a negative value on error.
int64_t synth_candidates(const uint8_t* genome, uint64_t G, const uint8_t* bases,
                         const int64_t* offsets, uint64_t n, uint32_t k, uint32_t bin_size,
                         uint32_t cap, int64_t* cand_off, int32_t* cand_bin) {
  if (k == 0 || k > 14 || bin_size == 0 || G < k) return -1;
  if (G > 0xFFFFFFFFull) return -3;  // positions are stored as uint32
  const uint64_t nk = 1ull << (2 * k);
  const uint64_t kmask = nk - 1;
  const int nth = omp_get_max_threads();
  // direct-address table: per-thread counts over contiguous genome ranges
  std::vector<uint64_t> start(nk + 1, 0);
  const uint64_t npos = G - k + 1;
  std::vector<std::vector<uint32_t>> tcount(nth);
  std::vector<uint64_t> lo(nth + 1);
  for (int t = 0; t <= nth; ++t) lo[t] = npos * (uint64_t)t / (uint64_t)nth;
#pragma omp parallel num_threads(nth)
  {
    int t = omp_get_thread_num();
    tcount[t].assign(nk, 0);
    uint64_t code = 0; uint32_t valid = 0;
    uint64_t s0 = lo[t];
    for (uint64_t i = s0; i < lo[t + 1] + k - 1 && i < G; ++i) {
      int c = code_of(genome[i]);
      if (c < 0) { valid = 0; code = 0; continue; }
      code = ((code << 2) | (uint64_t)c) & kmask;
      if (++valid >= k && i + 1 >= s0 + k) tcount[t][code]++;
    }
  }
  // prefix over (kmer, thread)
  std::vector<uint64_t> tbase((size_t)nth * nk);
  uint64_t acc = 0;
  for (uint64_t m = 0; m < nk; ++m) {
    start[m] = acc;
    for (int t = 0; t < nth; ++t) { tbase[(size_t)t * nk + m] = acc; acc += tcount[t][m]; }
  }
  start[nk] = acc;
  std::vector<uint32_t> posv(acc > 0 ? acc : 1);
  uint32_t* pos = posv.data();
#pragma omp parallel num_threads(nth)
  {
    int t = omp_get_thread_num();
    tcount[t].clear(); tcount[t].shrink_to_fit();
    uint64_t* tb = &tbase[(size_t)t * nk];
    uint64_t code = 0; uint32_t valid = 0;
    uint64_t s0 = lo[t];
    for (uint64_t i = s0; i < lo[t + 1] + k - 1 && i < G; ++i) {
      int c = code_of(genome[i]);
      if (c < 0) { valid = 0; code = 0; continue; }
      code = ((code << 2) | (uint64_t)c) & kmask;
      if (++valid >= k && i + 1 >= s0 + k) pos[tb[code]++] = (uint32_t)(i + 1 - k);
    }
  }
  tbase.clear(); tbase.shrink_to_fit();
  // per-read candidates
  std::vector<uint32_t> cnt(n);
#pragma omp parallel
  {
    std::vector<int64_t> loc;
    std::vector<std::pair<uint32_t, int32_t>> ranked;  // (votes, bin)
#pragma omp for schedule(dynamic, 256)
    for (int64_t r = 0; r < (int64_t)n; ++r) {
      const uint8_t* rd = bases + offsets[r];
      const int64_t L = offsets[r + 1] - offsets[r];
      loc.clear();
      for (int64_t o = 0; o + (int64_t)k <= L; o += k) {
        uint64_t code = 0; bool ok = true;
        for (uint32_t j = 0; j < k; ++j) {
          int c = code_of(rd[o + j]);
          if (c < 0) { ok = false; break; }
          code = (code << 2) | (uint64_t)c;
        }
        if (!ok) continue;
        for (uint64_t h = start[code]; h < start[code + 1]; ++h) {
          int64_t l = (int64_t)pos[h] - o;
          if (l < 0) l = 0;
          loc.push_back(l / (int64_t)bin_size);
        }
      }
      std::sort(loc.begin(), loc.end());
      ranked.clear();
      for (size_t i = 0; i < loc.size();) {
        size_t j = i;
        while (j < loc.size() && loc[j] == loc[i]) ++j;
        ranked.emplace_back((uint32_t)(j - i), (int32_t)loc[i]);
        i = j;
      }
      if (ranked.size() > cap) {
        std::stable_sort(ranked.begin(), ranked.end(),
                         [](const std::pair<uint32_t, int32_t>& a, const std::pair<uint32_t, int32_t>& b) {
                           return a.first != b.first ? a.first > b.first : a.second < b.second;
                         });
        ranked.resize(cap);
        std::sort(ranked.begin(), ranked.end(),
                  [](const std::pair<uint32_t, int32_t>& a, const std::pair<uint32_t, int32_t>& b) {
                    return a.second < b.second;
                  });
      }
      int32_t* dst = cand_bin + (uint64_t)r * cap;
      for (size_t i = 0; i < ranked.size(); ++i) dst[i] = ranked[i].second;
      cnt[r] = (uint32_t)ranked.size();
    }
  }
  // compact in place into CSR order (reads in increasing order: dst <= src)
  int64_t off = 0;
  for (uint64_t r = 0; r < n; ++r) {
    cand_off[r] = off;
    int32_t* src = cand_bin + r * cap;
    if (cand_bin + off != src) std::memmove(cand_bin + off, src, (size_t)cnt[r] * sizeof(int32_t));
    off += cnt[r];
  }
  cand_off[n] = off;
  return off;
}

}  // extern "C"
