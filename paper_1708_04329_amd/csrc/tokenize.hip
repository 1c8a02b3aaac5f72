// Read tokenisation and per-read thresholds.
//
// Step 1 of the filter (paper Section 3): every token (q-gram) of a read is
// extracted. Token i of read r is the code of read[i .. i+q) with A=0, C=1,
// G=2, T=3 and the first base most significant; a window holding any other
// byte gets the code R4 = 4^q, which the scan kernels treat as "never
// present". The threshold T_r = (L_r - q + 1) - q * E_r (Section 3) and the
// error budget E_r = ceil(e_r * L_r) (Section 6, read-existence figure
// caption) are computed here too, one per read.
//
// Tokens are written as code << tok_shift (the scan kernel wants the LDS byte
// offset of the token's row, the candidate kernel the plain code).
//
// A wavefront tokenises eight reads at once: lane j < 8 validates read j and
// writes its threshold, then the 64 lanes walk the reads' padded token ranges
// as one flat range, eight consecutive tokens per lane and group. Each lane
// loads the q + 7 bases its eight tokens span, slides a 2q-bit window over
// them and writes the entries with two 16-byte stores. A read's range is a
// multiple of 8 tokens, so a group of eight never straddles two reads, and
// every base load lies inside the read (positions past its end count as
// non-ACGT without a load).

#include "grim_internal.h"

namespace grim {
namespace {

constexpr uint32_t kTokReads = 8;  // reads per wavefront

// Branch-free base code: with the case folded, d = byte - 0x60 is 1, 3, 7, 20
// for a, c, g, t (bits of 0x10008A); ((d >> 1) ^ (d >> 2)) & 3 maps those to
// 0, 1, 2, 3. Any other byte gives -1.
__device__ __forceinline__ int base_code(uint32_t b) {
  const uint32_t d = (b | 0x20u) - 0x60u;
  const bool ok = d < 32u && ((0x0010008Au >> d) & 1u);
  return ok ? (int)(((d >> 1) ^ (d >> 2)) & 3u) : -1;
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t v, uint32_t k) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)k);
}

template <int Q>
__global__ __launch_bounds__(256) void k_tokenize(TokArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t r0 = ((uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6)) * kTokReads;
  const uint64_t n_reads = a.dyn ? min(a.dyn->n_reads, a.n_reads) : a.n_reads;
  const uint64_t n_bases = a.dyn ? min(a.dyn->n_bases, a.n_bases) : a.n_bases;
  if (r0 >= n_reads) return;

  // per-read checks, budget and threshold (lane j holds read r0 + j)
  uint64_t o_read = 0;
  uint32_t ntok_read = 0, npad_read = 0;
  const uint64_t r = r0 + lane;
  if (lane < kTokReads && r < n_reads) {
    const int64_t o0 = a.offsets[r], o1 = a.offsets[r + 1];
    uint32_t err = 0;
    int64_t L = o1 - o0;
    if (o0 < 0 || o1 < o0 || (uint64_t)o1 > n_bases) { err |= ST_BAD_LENGTH; L = 0; }
    if (L < (int64_t)Q) err |= ST_BAD_LENGTH;
    const int64_t ntok = L >= (int64_t)Q ? L - Q + 1 : 0;
    if (ntok > 65535) err |= ST_TOO_LONG;
    if (ntok > (int64_t)a.max_tokens) err |= ST_COUNT_U8;
    uint64_t E;
    if (a.max_edits) E = a.max_edits[r];
    else {
      const uint64_t e = a.err_pm ? a.err_pm[r] : a.err_pm_all;
      E = ((uint64_t)L * e + 999u) / 1000u;
    }
    if (!(a.flags & GRIM_READS_ALLOW_SHORT_OVERLAP) && L + (int64_t)E - (int64_t)Q > (int64_t)a.overlap)
      err |= ST_OVERLAP;
    int64_t T = (L - (int64_t)Q + 1) - (int64_t)Q * (int64_t)E;
    if (T < -(1 << 30)) T = -(1 << 30);
    a.thr[r] = (int32_t)T;
    if (err) atomicOr(a.status, err);
    if (!(err & (ST_BAD_LENGTH | ST_TOO_LONG))) {
      o_read = (uint64_t)o0;
      ntok_read = (uint32_t)ntok;
      // padded to the next multiple of 32 strictly above the token count: the
      // scan folds the last partial block exactly and may read one block past
      // the full ones; candidate checks read whole groups of four up to the
      // count, so a multiple of 8 serves them
      npad_read = a.short_pad ? (ntok_read + 7u) & ~7u : (ntok_read / 32u + 1u) * 32u;
    }
  }

  // the eight reads' ranges, wave-uniform: read k covers flat tokens
  // [start[k], start[k + 1]); a rejected or absent read covers none
  uint32_t start[kTokReads + 1], ntok[kTokReads];
  const uint8_t* src[kTokReads];
  uint32_t* dst[kTokReads];
  start[0] = 0;
#pragma unroll
  for (uint32_t k = 0; k < kTokReads; ++k) {
    const uint64_t o = ((uint64_t)lane_u32((uint32_t)(o_read >> 32), k) << 32) | lane_u32((uint32_t)o_read, k);
    ntok[k] = lane_u32(ntok_read, k);
    start[k + 1] = start[k] + lane_u32(npad_read, k);
    src[k] = a.bases + o;
    dst[k] = a.tokens + token_base((int64_t)o, r0 + k);
  }
  const uint32_t total = start[kTokReads];
  constexpr uint32_t R4 = 1u << (2 * Q);
  constexpr uint32_t MASK = R4 - 1u;
  constexpr int TPG = 8;            // consecutive tokens per lane and group
  constexpr int NB = Q + TPG - 1;   // bases they span
  constexpr uint32_t kSpan = 64u * TPG;
  const uint32_t sh = a.tok_shift;

  for (uint32_t f0 = TPG * lane; f0 < total; f0 += 2u * kSpan) {
    // two groups per lane and step, their loads issued together
    uint32_t by[2][NB];
    uint32_t i[2], n[2];
    uint32_t* out[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t f = f0 + kSpan * h;
      const uint8_t* s = src[0];
      uint32_t* d = dst[0];
      uint32_t nt = ntok[0], st = 0;
#pragma unroll
      for (uint32_t k = 1; k < kTokReads; ++k)
        if (f >= start[k]) { s = src[k]; d = dst[k]; nt = ntok[k]; st = start[k]; }
      const bool live = f < total;
      i[h] = f - st;
      n[h] = live ? nt : 0u;
      out[h] = d + i[h];
      // bases i .. i + NB - 1; positions at or past the read's end (L = nt + Q - 1)
      // are not loaded, nor is anything for a group past the flat range
      const uint32_t lim = live ? nt + (Q - 1) : 0u;
#pragma unroll
      for (int m = 0; m < NB; ++m) by[h][m] = i[h] + m < lim ? (uint32_t)s[i[h] + m] : 0u;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (f0 + kSpan * h >= total) continue;
      uint32_t code = 0, v[TPG];
      int last_bad = -1;  // position of the latest non-ACGT base
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const int b = base_code(by[h][m]);
        code = ((code << 2) | (uint32_t)(b & 3)) & MASK;
        if (b < 0) last_bad = m;
        if (m >= Q - 1) {
          const int u = m - (Q - 1);  // token i + u spans bases u .. m
          v[u] = (i[h] + u < n[h] && last_bad < u) ? code : R4;
        }
      }
#pragma unroll
      for (int g = 0; g < TPG / 4; ++g)
        reinterpret_cast<uint4*>(out[h])[g] =
            make_uint4(v[4 * g] << sh, v[4 * g + 1] << sh, v[4 * g + 2] << sh, v[4 * g + 3] << sh);
    }
  }
}

// Token order for the all-bins scan's LDS reads. The sum over a read's tokens
// does not depend on their order, so each read's tokens are reordered in
// place: those whose tile row has the read index's parity first, the others
// after, each class in its original order. The scan's launch order puts a read
// of even index beside one of odd index (the length order alternates them),
// and the two share the bank pass of every LDS read: one takes a row of even
// index where the other takes a row of odd index for all but about
// |evens(a) - odds(b)| token positions, and rows of opposite parity lie in
// different halves of the LDS banks (128-byte rows). One wavefront per read;
// reads of more than 256 tokens keep the sequence order.
__global__ __launch_bounds__(256) void k_pair_order(TokArgs a) {
  const uint64_t r = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint64_t n_reads = a.dyn ? min(a.dyn->n_reads, a.n_reads) : a.n_reads;
  const uint64_t n_bases = a.dyn ? min(a.dyn->n_bases, a.n_bases) : a.n_bases;
  if (r >= n_reads) return;
  const int64_t o0 = a.offsets[r], o1 = a.offsets[r + 1];
  // the tokenizer flagged reads with bad offsets or lengths and wrote no entries
  if (o0 < 0 || o1 < o0 || (uint64_t)o1 > n_bases || o1 - o0 < (int64_t)a.q) return;
  const uint64_t ntok = (uint64_t)(o1 - o0) - a.q + 1;
  if (ntok > 256) return;
  uint32_t* t = a.tokens + token_base(o0, r);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t want = (uint32_t)(r & 1u);
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t v[4], first_before[4];
  bool first[4];
  uint32_t nfirst = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t p = lane + 64u * j;
    v[j] = p < ntok ? t[p] : 0u;
    first[j] = p < ntok && ((v[j] >> a.tok_shift) & 1u) == want;
    const uint64_t bal = __ballot(first[j]);
    first_before[j] = nfirst + (uint32_t)__popcll(bal & lt);
    nfirst += (uint32_t)__popcll(bal);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t p = lane + 64u * j;
    if (p < ntok) t[first[j] ? first_before[j] : nfirst + (p - first_before[j])] = v[j];
  }
}

}  // namespace

// With a.dyn set, a.n_reads / a.n_bases are the capacities the grid is sized for.
hipError_t launch_tokenize(const TokArgs& a, hipStream_t s) {
  if (a.n_reads == 0) return hipSuccess;
  // entries are written with 16-byte stores
  if (reinterpret_cast<uintptr_t>(a.tokens) & 15u) return hipErrorInvalidValue;
  const uint64_t reads_per_block = 4ull * kTokReads;
  const uint64_t blocks = (a.n_reads + reads_per_block - 1) / reads_per_block;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)blocks), block(256);
  switch (a.q) {
    case 1: hipLaunchKernelGGL(k_tokenize<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_tokenize<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_tokenize<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_tokenize<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_tokenize<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_tokenize<6>, grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_tokenize<7>, grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_tokenize<8>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.pair_order) return e;
  const uint64_t pblocks = (a.n_reads + 3) / 4;
  if (pblocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_pair_order, dim3((unsigned)pblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace grim
