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
// Work split: one lane per pair. A first pass counts the pairs to align per
// read length class (words per read, 1..16) and writes the outputs of the
// pairs it skips; a second pass lists the pairs class by class, so that one
// launch per class runs lanes with equal word counts in lock step.

#include "grim_internal.h"

namespace grim {
namespace {

constexpr uint32_t kSkipped = 0xFFFFu;

__global__ __launch_bounds__(256) void k_verify_count(VerifyArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t r = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.n_reads) return;
  if (a.status[0] & ~(uint32_t)(ST_BAD_BIN | ST_BAD_CAND_OFF | ST_VERIFY_LONG)) return;  // rejected reads
  const int64_t c0 = a.cand_off[r], c1 = a.cand_off[r + 1];
  if (c0 < 0 || c1 < c0 || (uint64_t)c1 > a.n_cand) {
    if (lane == 0) atomicOr(a.status, ST_BAD_CAND_OFF);
    return;
  }
  const uint64_t L = (uint64_t)(a.offsets[r + 1] - a.offsets[r]);
  uint64_t n_sel = 0;
  for (int64_t k0 = c0; k0 < c1; k0 += 64) {
    const int64_t k = k0 + lane;
    bool sel = false;
    if (k < c1) {
      const int32_t x = a.cand_bin[k];
      if (x < 0 || (uint64_t)x >= a.nb) atomicOr(a.status, ST_BAD_BIN);
      else sel = !a.verify_mask || a.verify_mask[k];
      if (!sel) {
        a.dist_out[k] = (uint16_t)kSkipped;
        a.match_out[k] = 0;
      }
    }
    n_sel += (uint64_t)__popcll(__ballot(sel));
  }
  if (n_sel == 0 || lane != 0) return;
  if (L > kVerifyMaxLen || L == 0) {
    atomicOr(a.status, ST_VERIFY_LONG);
    return;
  }
  atomicAdd(reinterpret_cast<unsigned long long*>(a.bucket + (L + 31) / 32), (unsigned long long)n_sel);
}

__global__ __launch_bounds__(256) void k_verify_scatter(VerifyArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t r = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.n_reads) return;
  const int64_t c0 = a.cand_off[r], c1 = a.cand_off[r + 1];
  const uint64_t L = (uint64_t)(a.offsets[r + 1] - a.offsets[r]);
  if (L == 0 || L > kVerifyMaxLen) return;
  unsigned long long* cursor = reinterpret_cast<unsigned long long*>(a.bucket + (L + 31) / 32);
  for (int64_t k0 = c0; k0 < c1; k0 += 64) {
    const int64_t k = k0 + lane;
    bool sel = false;
    if (k < c1) {
      const int32_t x = a.cand_bin[k];
      sel = x >= 0 && (uint64_t)x < a.nb && (!a.verify_mask || a.verify_mask[k]);
    }
    const uint64_t m = __ballot(sel);
    if (m == 0) continue;
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd(cursor, (unsigned long long)__popcll(m));
    base = ((uint64_t)(uint32_t)__shfl((int)(base >> 32), 0) << 32) | (uint32_t)__shfl((int)(uint32_t)base, 0);
    if (sel) {
      const uint64_t below = m & ((1ull << lane) - 1ull);
      const uint64_t pos = base + (uint64_t)__popcll(below);
      a.item_pair[pos] = (uint64_t)k;
      a.item_read[pos] = (uint32_t)r;
    }
  }
}

// Myers' column step for W words. pe[c][w]: bit i of word w set when read
// base 32w + i has code c. pv/mv: vertical +1/-1 bits of the current column.
// `top` is the read's last row within word W - 1; `score` tracks that row.
template <int W>
struct Column {
  uint32_t pe[4][W];
  uint32_t pv[W], mv[W];
  uint32_t top;
  int32_t score, best;

  __device__ __forceinline__ void step(uint32_t c) {
    const uint32_t valid = c < 4u ? 0xFFFFFFFFu : 0u;  // other bytes match nothing
    const bool odd = (c & 1u) != 0, high = (c & 2u) != 0;
    uint32_t hp = 0, hm = 0;  // horizontal difference entering word w's bottom row
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t ac = odd ? pe[1][w] : pe[0][w];
      const uint32_t gt = odd ? pe[3][w] : pe[2][w];
      uint32_t eq = (high ? gt : ac) & valid;
      const uint32_t xv = eq | mv[w];
      eq |= hm;  // a -1 entering from below acts as a match in the carry chain
      const uint32_t xh = (((eq & pv[w]) + pv[w]) ^ pv[w]) | eq;
      uint32_t ph = mv[w] | ~(xh | pv[w]);
      uint32_t mh = pv[w] & xh;
      if (w == W - 1) score += (int32_t)((ph >> top) & 1u) - (int32_t)((mh >> top) & 1u);
      const uint32_t hp_out = ph >> 31, hm_out = mh >> 31;
      ph = (ph << 1) | hp;
      mh = (mh << 1) | hm;
      pv[w] = mh | ~(xv | ph);
      mv[w] = ph & xv;
      hp = hp_out;
      hm = hm_out;
    }
    best = min(best, score);
  }
};

template <int W>
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

  Column<W> col;
  const uint8_t* rd = a.bases + o0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    for (uint32_t b = 0; b < 32; ++b) {
      const uint32_t i = (uint32_t)w * 32 + b;
      if (i >= L) break;
      const uint32_t c = rd[i] | 0x20u;  // fold ASCII letters to lower case
      const uint32_t bit = 1u << b;
      m0 |= c == 'a' ? bit : 0u;
      m1 |= c == 'c' ? bit : 0u;
      m2 |= c == 'g' ? bit : 0u;
      m3 |= c == 't' ? bit : 0u;
    }
    col.pe[0][w] = m0;
    col.pe[1][w] = m1;
    col.pe[2][w] = m2;
    col.pe[3][w] = m3;
    col.pv[w] = 0xFFFFFFFFu;  // column 0: row i holds distance i
    col.mv[w] = 0;
  }
  col.top = (L - 1) & 31u;
  col.score = (int32_t)L;
  col.best = (int32_t)L;

  const uint8_t* txt = a.ref;
  uint64_t j = lo;
  const uint64_t aligned = min(hi, (lo + 15) & ~15ull);
  for (; j < aligned; ++j) col.step(txt[j]);
  for (; j + 16 <= hi; j += 16) {
    const uint4 v = *reinterpret_cast<const uint4*>(txt + j);
    const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
      for (int by = 0; by < 4; ++by) col.step((wv[q4] >> (8 * by)) & 0xFFu);
  }
  for (; j < hi; ++j) col.step(txt[j]);

  const int32_t T = a.thr[r];
  const int64_t E = ((int64_t)L - (int64_t)a.q + 1 - (int64_t)T) / (int64_t)a.q;
  const uint32_t d = (uint32_t)min(col.best, (int32_t)0xFFFE);
  a.dist_out[k] = (uint16_t)d;
  a.match_out[k] = (int64_t)d <= E ? 1 : 0;
}

template <int W>
hipError_t launch_align_w(const VerifyArgs& a, uint64_t first, uint64_t count, hipStream_t s) {
  const uint64_t blocks = (count + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_verify_align<W>, dim3((unsigned)blocks), dim3(256), 0, s, a, first, count);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_verify_count(const VerifyArgs& a, hipStream_t s) {
  const uint64_t blocks = (a.n_reads + 3) / 4;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_verify_count, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_verify_scatter(const VerifyArgs& a, hipStream_t s) {
  const uint64_t blocks = (a.n_reads + 3) / 4;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_verify_scatter, dim3((unsigned)blocks), dim3(256), 0, s, a);
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
