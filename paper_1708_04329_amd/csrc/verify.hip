// Verification of filtered locations: the alignment step that follows the
// filter in a seed-and-extend mapper (paper Section 1, step 5; Section 5
// counts a passing location that yields no mapping against the filter).
//
// For a (read, bin) pair the result is the smallest Levenshtein distance
// between the whole read and any substring of the bases bin x's tokens cover,
// [x*B, min(x*B + B + O + q - 1, G)). It is computed with Myers' bit-vector
// algorithm (G. Myers, "A fast bit-vector algorithm for approximate string
// matching based on dynamic programming", J. ACM 46(3), 1999): one column of
// the dynamic-programming matrix is held as vertical +1/-1 difference bits,
// 32 rows per uint32 word, and each reference base advances every word with
// a dozen bitwise operations and one add. Reads longer than 32 bases use
// Myers' block form: word w hands its top row's horizontal difference to
// word w + 1. Row 0 has horizontal difference 0 in every column, so an
// alignment may start anywhere in the text, and the distance is the minimum
// over all columns of the last row.
//
// The read's match masks are kept as two code bit planes and a validity
// plane, so a text base selects its mask with two three-input operations
// per word; 16-byte text chunks holding a byte other than A, C, G, T (N
// runs) take a checked step that masks it out.
//
// Work split: one lane per pair. A first pass counts the pairs to align per
// read length class (words per read, 1..16) and writes the outputs of the
// pairs it skips; a prefix over chunks of reads turns the counts into list
// positions (no global atomics, which would serialise on a few class
// counters); a second pass lists the pairs class by class, so that one
// launch per class runs lanes with equal word counts in lock step.

#include <type_traits>

#include "grim_internal.h"

namespace grim {
namespace {

constexpr uint32_t kSkipped = 0xFFFFu;
constexpr int kGroups = 16;

// Selection of pair k: a valid bin, and the mask (if any) set.
__device__ __forceinline__ bool selected(const VerifyArgs& a, int32_t x, uint8_t m) {
  return x >= 0 && (uint64_t)x < a.nb && (!a.verify_mask || m);
}

// Bin ids and mask bytes of kGroups consecutive 64-pair groups from k0, all
// loads issued before the first wait (past the end: the read's last pair,
// ignored by the caller).
__device__ __forceinline__ void load_groups(const VerifyArgs& a, int64_t k0, int64_t c1, uint32_t lane,
                                            int32_t (&x)[kGroups], uint8_t (&m)[kGroups]) {
#pragma unroll
  for (int u = 0; u < kGroups; ++u) x[u] = a.cand_bin[min(k0 + u * 64 + (int64_t)lane, c1 - 1)];
  if (a.verify_mask) {
#pragma unroll
    for (int u = 0; u < kGroups; ++u) m[u] = a.verify_mask[min(k0 + u * 64 + (int64_t)lane, c1 - 1)];
  } else {
#pragma unroll
    for (int u = 0; u < kGroups; ++u) m[u] = 1;
  }
}

__device__ __forceinline__ uint32_t length_class(const VerifyArgs& a, uint64_t r) {
  const uint64_t L = (uint64_t)(a.offsets[r + 1] - a.offsets[r]);
  return (L == 0 || L > kVerifyMaxLen) ? 0u : (uint32_t)((L + 31) / 32);
}

// First pass, one workgroup of 16 wavefronts per chunk of kVerifyChunk reads,
// a wavefront per read: count the read's selected pairs (read_sel), write the outputs of the
// pairs it skips, and sum the counts per length class for the chunk
// (chunk_sum[chunk][class]). No global atomics: the list positions come from
// a prefix over chunks.
__global__ __launch_bounds__(1024) void k_verify_count(VerifyArgs a) {
  __shared__ unsigned long long csum[kVerifyBuckets];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  if (threadIdx.x < kVerifyBuckets) csum[threadIdx.x] = 0;
  __syncthreads();
  const bool rejected = a.status[0] & ~(uint32_t)(ST_BAD_BIN | ST_BAD_CAND_OFF | ST_VERIFY_LONG);
  const uint64_t r_lo = (uint64_t)blockIdx.x * kVerifyChunk;
  const uint64_t r_hi = min(a.n_reads, r_lo + kVerifyChunk);
  for (uint64_t r = r_lo + wave; r < r_hi && !rejected; r += 16) {
    const int64_t c0 = a.cand_off[r], c1 = a.cand_off[r + 1];
    if (c0 < 0 || c1 < c0 || (uint64_t)c1 > a.n_cand || c1 - c0 > 0xFFFFFFFFll) {
      if (lane == 0) {
        atomicOr(a.status, ST_BAD_CAND_OFF);
        a.read_sel[r] = 0;
      }
      continue;
    }
    uint32_t n_sel = 0;
    for (int64_t k0 = c0; k0 < c1; k0 += kGroups * 64) {
      int32_t x[kGroups];
      uint8_t m[kGroups];
      load_groups(a, k0, c1, lane, x, m);
#pragma unroll
      for (int u = 0; u < kGroups; ++u) {
        const int64_t k = k0 + u * 64 + lane;
        bool sel = false;
        if (k < c1) {
          if (x[u] < 0 || (uint64_t)x[u] >= a.nb) atomicOr(a.status, ST_BAD_BIN);
          sel = selected(a, x[u], m[u]);
          if (!sel) {
            a.dist_out[k] = (uint16_t)kSkipped;
            a.match_out[k] = 0;
          }
        }
        n_sel += (uint32_t)__popcll(__ballot(sel));
      }
    }
    if (lane == 0) {
      a.read_sel[r] = n_sel;
      if (n_sel) {
        const uint32_t cls = length_class(a, r);
        if (cls == 0) atomicOr(a.status, ST_VERIFY_LONG);
        else atomicAdd(&csum[cls], (unsigned long long)n_sel);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kVerifyBuckets) a.chunk_sum[(uint64_t)blockIdx.x * kVerifyBuckets + threadIdx.x] = csum[threadIdx.x];
}

// One wavefront per length class 1..16 (class 0 holds no pairs): a scan
// over the chunks, 64 at a time, turns chunk_sum[chunk][class] into the list
// slot of the chunk's first pair of that class; bucket[class] gets the
// class's pair count (the host launches one alignment per class). Classes
// follow each other in the list in increasing order.
__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, uint32_t d) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, d), hi = (uint32_t)__shfl_up((int)(v >> 32), d);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(1024) void k_verify_prefix(VerifyArgs a, uint64_t n_chunks) {
  __shared__ unsigned long long total[kVerifyBuckets];
  const uint32_t lane = threadIdx.x & 63u, c = 1 + (threadIdx.x >> 6);  // classes 1..16
  unsigned long long acc = 0;
  for (uint64_t k0 = 0; k0 < n_chunks; k0 += 64) {
    const uint64_t k = k0 + lane;
    const uint64_t v = k < n_chunks ? a.chunk_sum[k * kVerifyBuckets + c] : 0;
    uint64_t incl = v;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
      const uint64_t t = shfl_up64(incl, d);
      if (lane >= d) incl += t;
    }
    if (k < n_chunks) a.chunk_sum[k * kVerifyBuckets + c] = acc + incl - v;
    const uint64_t sum64 = ((uint64_t)(uint32_t)__shfl((int)(incl >> 32), 63) << 32) |
                           (uint32_t)__shfl((int)(uint32_t)incl, 63);
    acc += sum64;
  }
  if (lane == 0) total[c] = acc;
  if (threadIdx.x == 0) total[0] = 0;
  __syncthreads();
  unsigned long long first = 0;
  for (uint32_t i = 0; i < c; ++i) first += total[i];
  for (uint64_t k = lane; k < n_chunks; k += 64) a.chunk_sum[k * kVerifyBuckets + c] += first;
  if (lane == 0) a.bucket[c] = acc;
  if (threadIdx.x == 0) a.bucket[0] = 0;
}

// Second pass, same chunks: the reads' first slots, in read order within each
// class (one thread per class over the chunk), then each wavefront lists its
// read's selected pairs in pair order.
__global__ __launch_bounds__(1024) void k_verify_scatter(VerifyArgs a) {
  __shared__ unsigned long long base[kVerifyChunk];
  __shared__ uint32_t sel_s[kVerifyChunk];
  __shared__ uint8_t cls_s[kVerifyChunk];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint64_t r_lo = (uint64_t)blockIdx.x * kVerifyChunk;
  const uint64_t r_hi = min(a.n_reads, r_lo + kVerifyChunk);
  const uint32_t n = (uint32_t)(r_hi - r_lo);
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    sel_s[i] = a.read_sel[r_lo + i];
    cls_s[i] = (uint8_t)length_class(a, r_lo + i);
  }
  __syncthreads();
  if (threadIdx.x < kVerifyBuckets) {
    unsigned long long cur = a.chunk_sum[(uint64_t)blockIdx.x * kVerifyBuckets + threadIdx.x];
    for (uint32_t i = 0; i < n; ++i) {
      if (cls_s[i] != threadIdx.x) continue;
      base[i] = cur;
      cur += sel_s[i];
    }
  }
  __syncthreads();
  for (uint64_t r = r_lo + wave; r < r_hi; r += 16) {
    const uint32_t i = (uint32_t)(r - r_lo);
    if (sel_s[i] == 0 || cls_s[i] == 0) continue;
    const int64_t c0 = a.cand_off[r], c1 = a.cand_off[r + 1];
    uint64_t pos0 = base[i];
    for (int64_t k0 = c0; k0 < c1; k0 += kGroups * 64) {
      int32_t x[kGroups];
      uint8_t m[kGroups];
      load_groups(a, k0, c1, lane, x, m);
#pragma unroll
      for (int u = 0; u < kGroups; ++u) {
        const int64_t k = k0 + u * 64 + lane;
        const bool sel = k < c1 && selected(a, x[u], m[u]);
        const uint64_t bal = __ballot(sel);
        if (sel) {
          const uint64_t pos = pos0 + (uint64_t)__popcll(bal & ((1ull << lane) - 1ull));
          a.item_pair[pos] = (uint64_t)k;
          a.item_read[pos] = (uint32_t)r;
        }
        pos0 += (uint64_t)__popcll(bal);
      }
    }
  }
}

// Myers' column step for W words. The read is held as bit planes: bit i of
// word w of r0 / r1 is bit 0 / bit 1 of the code of read base 32w + i, and
// va marks the bases that are A, C, G or T; so the match mask of text code c
// is va & ~(r0 ^ c0) & ~(r1 ^ c1) with c0, c1 the bits of c spread to all
// 32 positions, two three-input operations per word. pv/mv: vertical +1/-1
// bits of the current column; `top` is the read's last row within word
// W - 1, whose distance `score` tracks. CHECKED steps also accept text bytes
// other than 0..3 (they match nothing).
template <int W>
struct Column {
  uint32_t r0[W], r1[W], va[W];
  uint32_t pv[W], mv[W];
  uint32_t top;
  int32_t score, best;

  template <bool CHECKED>
  __device__ __forceinline__ void step(uint32_t c) {
    const uint32_t c0 = 0u - (c & 1u), c1 = 0u - ((c >> 1) & 1u);
    const uint32_t valid = (!CHECKED || c < 4u) ? 0xFFFFFFFFu : 0u;
    // the previous word's unshifted horizontal +1/-1 bits: their top bit is
    // the difference entering this word's bottom row (0 below word 0)
    uint32_t php = 0, mhp = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      // truth tables of bitop3 over (src0, src1, src2) = 0xF0, 0xCC, 0xAA
      uint32_t eq = __builtin_amdgcn_bitop3_b32(va[w], r0[w], c0, 0x90);  // va & ~(r0 ^ c0)
      eq = __builtin_amdgcn_bitop3_b32(eq, r1[w], c1, 0x90);              //    & ~(r1 ^ c1)
      if (CHECKED) eq &= valid;
      const uint32_t xv = eq | mv[w];
      eq |= mhp >> 31;  // a -1 entering from below acts as a match in the carry chain
      const uint32_t sum = (eq & pv[w]) + pv[w];
      const uint32_t xh = __builtin_amdgcn_bitop3_b32(sum, pv[w], eq, 0xBE);  // (sum ^ pv) | eq
      const uint32_t ph = mv[w] | ~(xh | pv[w]);
      const uint32_t mh = pv[w] & xh;
      if (w == W - 1) score += (int32_t)((ph >> top) & 1u) - (int32_t)((mh >> top) & 1u);
      // shift up one row, the entering difference moving into row 0
      const uint32_t phs = __builtin_amdgcn_alignbit(ph, php, 31);
      const uint32_t mhs = __builtin_amdgcn_alignbit(mh, mhp, 31);
      pv[w] = mhs | ~(xv | phs);
      mv[w] = phs & xv;
      php = ph;
      mhp = mh;
    }
    best = min(best, score);
  }
};

// Bounded form of the same step (Myers 1999, Section 4: the block-based
// algorithm with Ukkonen's cutoff): only words 0..y advance, y being the last
// word that can hold a distance <= k in this column; every cell below it is
// known to exceed k. sc[w] is the distance at word w's last row (row `top`
// for word W - 1). Word y + 1 joins when its first row can reach k: the last
// active word's bottom was <= k in the previous column and either the text
// base matches that first row or the bottom decreased. It joins as if its
// previous column rose by one per row (Myers' initialisation; cells whose
// true distance is <= k still come out exact). A last active word leaves once
// its last row's distance minus its +1 bits exceeds k (no cell of it can then
// be <= k). Distances <= k are exact; larger ones are reported as k + 1.
template <int W>
struct ColumnB {
  uint32_t r0[W], r1[W], va[W];
  uint32_t pv[W], mv[W];
  int32_t sc[W];
  uint32_t top, lastmask;  // lastmask: rows 0..top of word W - 1
  int32_t k, y, best;

  template <bool CHECKED>
  __device__ __forceinline__ void step(uint32_t c) {
    const uint32_t c0 = 0u - (c & 1u), c1 = 0u - ((c >> 1) & 1u);
    const uint32_t valid = (!CHECKED || c < 4u) ? 0xFFFFFFFFu : 0u;
    uint32_t php = 0, mhp = 0;
    int32_t hprev = 0;  // horizontal difference out of the previous word's last row
    int32_t yn = y;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint32_t eq = __builtin_amdgcn_bitop3_b32(va[w], r0[w], c0, 0x90);
      eq = __builtin_amdgcn_bitop3_b32(eq, r1[w], c1, 0x90);
      if (CHECKED) eq &= valid;
      if (w > 0 && w == yn + 1 && sc[w - 1] - hprev <= k && ((eq & 1u) || hprev < 0)) {
        pv[w] = 0xFFFFFFFFu;
        mv[w] = 0;
        sc[w] = sc[w - 1] - hprev + (w == W - 1 ? (int32_t)top + 1 : 32);
        yn = w;
      }
      if (w <= yn) {
        const uint32_t xv = eq | mv[w];
        eq |= mhp >> 31;
        const uint32_t sum = (eq & pv[w]) + pv[w];
        const uint32_t xh = __builtin_amdgcn_bitop3_b32(sum, pv[w], eq, 0xBE);  // (sum ^ pv) | eq
        const uint32_t ph = mv[w] | ~(xh | pv[w]);
        const uint32_t mh = pv[w] & xh;
        const uint32_t bit = w == W - 1 ? top : 31u;
        hprev = (int32_t)((ph >> bit) & 1u) - (int32_t)((mh >> bit) & 1u);
        sc[w] += hprev;
        const uint32_t phs = __builtin_amdgcn_alignbit(ph, php, 31);
        const uint32_t mhs = __builtin_amdgcn_alignbit(mh, mhp, 31);
        pv[w] = mhs | ~(xv | phs);
        mv[w] = phs & xv;
        php = ph;
        mhp = mh;
      }
    }
    y = yn;
    if (y == W - 1) best = min(best, sc[W - 1]);
    // going up from a word's last row the distance falls by at most one per
    // +1 bit, so a last active word whose last row minus its +1 bits exceeds
    // k holds no cell <= k and leaves
#pragma unroll
    for (int w = W - 1; w >= 1; --w)
      if (y == w && sc[w] - (int32_t)__popc(w == W - 1 ? pv[w] & lastmask : pv[w]) > k) y = w - 1;
  }
};

template <int W, bool BOUNDED>
__global__ __launch_bounds__(256) void k_verify_align(VerifyArgs a, uint64_t first, uint64_t count) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint64_t k = a.item_pair[first + t];
  const uint32_t r = a.item_read[first + t];
  const int64_t o0 = a.offsets[r];
  const uint32_t L = (uint32_t)(a.offsets[r + 1] - o0);
  const uint64_t x = (uint64_t)a.cand_bin[k];

  // the bases bin x's tokens cover
  const uint64_t starts_end = a.G >= a.q ? a.G - a.q + 1 : 0;
  uint64_t lo = x * a.B, hi = lo + a.B + a.O;
  if (hi > starts_end) hi = starts_end;
  if (lo > hi) lo = hi;
  hi = hi > lo ? hi + a.q - 1 : lo;

  // the read's error budget, recovered from its threshold
  const int32_t T = a.thr[r];
  const int64_t E = ((int64_t)L - (int64_t)a.q + 1 - (int64_t)T) / (int64_t)a.q;
  using Col = typename std::conditional<BOUNDED, ColumnB<W>, Column<W>>::type;
  Col col;
  const uint8_t* rd = a.bases + o0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint32_t b0 = 0, b1 = 0, ok = 0;
    for (uint32_t b = 0; b < 32; ++b) {
      const uint32_t i = (uint32_t)w * 32 + b;
      if (i >= L) break;
      const uint32_t ch = rd[i] | 0x20u;  // fold ASCII letters to lower case
      const uint32_t code = ch == 'a' ? 0u : ch == 'c' ? 1u : ch == 'g' ? 2u : ch == 't' ? 3u : 4u;
      const uint32_t bit = 1u << b;
      b0 |= (code & 1u) ? bit : 0u;
      b1 |= (code & 2u) ? bit : 0u;
      ok |= code < 4u ? bit : 0u;
    }
    col.r0[w] = b0;
    col.r1[w] = b1;
    col.va[w] = ok;
    col.pv[w] = 0xFFFFFFFFu;  // column 0: row i holds distance i
    col.mv[w] = 0;
  }
  col.top = (L - 1) & 31u;
  col.best = (int32_t)L;
  if constexpr (BOUNDED) {
    // column 0: row i holds distance i + 1, so the words up to the one holding
    // row k - 1 start active (word 0 always)
    col.k = (int32_t)min<int64_t>(E, 1 << 20);
    col.lastmask = col.top == 31u ? 0xFFFFFFFFu : (2u << col.top) - 1u;
    col.y = col.k >= 1 ? min((int32_t)W - 1, (col.k - 1) / 32) : 0;
#pragma unroll
    for (int w = 0; w < W; ++w) col.sc[w] = w == W - 1 ? (int32_t)L : 32 * (w + 1);
  } else {
    col.score = (int32_t)L;
  }

  const uint8_t* txt = a.ref;
  uint64_t j = lo;
  const uint64_t aligned = min(hi, (lo + 15) & ~15ull);
  for (; j < aligned; ++j) col.template step<true>(txt[j]);
  for (; j + 16 <= hi; j += 16) {
    const uint4 v = *reinterpret_cast<const uint4*>(txt + j);
    const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
    if (((v.x | v.y | v.z | v.w) & 0xFCFCFCFCu) == 0) {  // A, C, G, T only (the common case)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
        for (int by = 0; by < 4; ++by) col.template step<false>((wv[q4] >> (8 * by)) & 0xFFu);
    } else {
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
        for (int by = 0; by < 4; ++by) col.template step<true>((wv[q4] >> (8 * by)) & 0xFFu);
    }
  }
  for (; j < hi; ++j) col.template step<true>(txt[j]);

  uint32_t d = (uint32_t)min(col.best, (int32_t)0xFFFE);
  if (a.bounded && (int64_t)d > E) d = (uint32_t)min<int64_t>(E + 1, 0xFFFE);  // the bounded output
  a.dist_out[k] = (uint16_t)d;
  a.match_out[k] = (int64_t)d <= E ? 1 : 0;
}

template <int W>
hipError_t launch_align_w(const VerifyArgs& a, uint64_t first, uint64_t count, hipStream_t s) {
  const uint64_t blocks = (count + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  // the cutoff pays off for reads of up to 6 words (measured: 1.3x at 4 and 5
  // words, 0.86x at 8, where lanes diverge over more words); longer reads run
  // the full column and cap the distance
  if (a.bounded && W <= 6)
    hipLaunchKernelGGL((k_verify_align<W, true>), dim3((unsigned)blocks), dim3(256), 0, s, a, first, count);
  else
    hipLaunchKernelGGL((k_verify_align<W, false>), dim3((unsigned)blocks), dim3(256), 0, s, a, first, count);
  return hipGetLastError();
}

}  // namespace

uint64_t verify_chunks(uint64_t n_reads) { return (n_reads + kVerifyChunk - 1) / kVerifyChunk; }

hipError_t launch_verify_count(const VerifyArgs& a, hipStream_t s) {
  const uint64_t chunks = verify_chunks(a.n_reads);
  if (chunks == 0) return hipSuccess;
  if (chunks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_verify_count, dim3((unsigned)chunks), dim3(1024), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_verify_prefix, dim3(1), dim3(1024), 0, s, a, chunks);
  return hipGetLastError();
}

hipError_t launch_verify_scatter(const VerifyArgs& a, hipStream_t s) {
  const uint64_t chunks = verify_chunks(a.n_reads);
  if (chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_verify_scatter, dim3((unsigned)chunks), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_verify_align(const VerifyArgs& a, uint32_t words, uint64_t first, uint64_t count,
                               hipStream_t s) {
  if (count == 0) return hipSuccess;
  switch (words) {
    case 1: return launch_align_w<1>(a, first, count, s);
    case 2: return launch_align_w<2>(a, first, count, s);
    case 3: return launch_align_w<3>(a, first, count, s);
    case 4: return launch_align_w<4>(a, first, count, s);
    case 5: return launch_align_w<5>(a, first, count, s);
    case 6: return launch_align_w<6>(a, first, count, s);
    case 7: return launch_align_w<7>(a, first, count, s);
    case 8: return launch_align_w<8>(a, first, count, s);
    case 9: return launch_align_w<9>(a, first, count, s);
    case 10: return launch_align_w<10>(a, first, count, s);
    case 11: return launch_align_w<11>(a, first, count, s);
    case 12: return launch_align_w<12>(a, first, count, s);
    case 13: return launch_align_w<13>(a, first, count, s);
    case 14: return launch_align_w<14>(a, first, count, s);
    case 15: return launch_align_w<15>(a, first, count, s);
    case 16: return launch_align_w<16>(a, first, count, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace grim
