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
// One wavefront per read: lane l writes tokens l, l + 64, ... so stores are
// coalesced; each token re-reads its q bases, which stay in L1/L2.

#include "grim_internal.h"

namespace grim {
namespace {

__device__ __forceinline__ int base_code(uint32_t b) {
  const uint32_t u = b | 0x20u;  // fold case
  if (u == 'a') return 0;
  if (u == 'c') return 1;
  if (u == 'g') return 2;
  if (u == 't') return 3;
  return -1;
}

__global__ __launch_bounds__(256) void k_tokenize(TokArgs a) {
  const uint64_t r = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t n_reads = a.dyn ? min(a.dyn->n_reads, a.n_reads) : a.n_reads;
  const uint64_t n_bases = a.dyn ? min(a.dyn->n_bases, a.n_bases) : a.n_bases;
  if (r >= n_reads) return;
  const int64_t o0 = a.offsets[r], o1 = a.offsets[r + 1];
  uint32_t err = 0;
  int64_t L = o1 - o0;
  if (o0 < 0 || o1 < o0 || (uint64_t)o1 > n_bases) { err |= ST_BAD_LENGTH; L = 0; }
  const uint32_t q = a.q;
  if (L < (int64_t)q) err |= ST_BAD_LENGTH;
  const int64_t ntok = L >= (int64_t)q ? L - q + 1 : 0;
  if (ntok > 65535) err |= ST_TOO_LONG;
  if (ntok > (int64_t)a.max_tokens) err |= ST_COUNT_U8;
  uint64_t E;
  if (a.max_edits) E = a.max_edits[r];
  else {
    const uint64_t e = a.err_pm ? a.err_pm[r] : a.err_pm_all;
    E = ((uint64_t)L * e + 999u) / 1000u;
  }
  if (!(a.flags & GRIM_READS_ALLOW_SHORT_OVERLAP) && L + (int64_t)E - (int64_t)q > (int64_t)a.overlap)
    err |= ST_OVERLAP;
  if (lane == 0) {
    int64_t T = (L - (int64_t)q + 1) - (int64_t)q * (int64_t)E;
    if (T < -(1 << 30)) T = -(1 << 30);
    a.thr[r] = (int32_t)T;
    if (err) atomicOr(a.status, err);
  }
  if (err & (ST_BAD_LENGTH | ST_TOO_LONG)) return;
  const uint32_t R4 = 1u << (2 * q);
  const uint8_t* rd = a.bases + o0;
  uint32_t* out = a.tokens + token_base(o0, r);
  // pad to the next multiple of 32 strictly above ntok: the scan folds the
  // last partial block exactly and may read one block past the full ones
  const int64_t npad = (ntok / 32 + 1) * 32;
  for (int64_t i = lane; i < npad; i += 64) {
    uint32_t code = R4;
    if (i < ntok) {
      uint32_t c = 0;
      bool ok = true;
      for (uint32_t j = 0; j < q; ++j) {
        const int b = base_code(rd[i + j]);
        ok = ok && b >= 0;
        c = (c << 2) | (uint32_t)(b & 3);
      }
      if (ok) code = c;
    }
    out[i] = code << a.tok_shift;
  }
}

}  // namespace

// With a.dyn set, a.n_reads / a.n_bases are the capacities the grid is sized for.
hipError_t launch_tokenize(const TokArgs& a, hipStream_t s) {
  if (a.n_reads == 0) return hipSuccess;
  const uint64_t blocks = (a.n_reads + 3) / 4;
  hipLaunchKernelGGL(k_tokenize, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace grim
