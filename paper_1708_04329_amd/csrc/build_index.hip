// Bit-vector generation (paper Section 3): the reference is scanned once;
// a token whose first base s lies in the extent [x*B, x*B + B + O) of bin x
// (and s <= G - q) sets bit t of bin x. The same bits are laid out two ways:
//
//   token-major (TM): row t holds bit x of every bin, rows padded to a
//     multiple of 64 words. One row read gives one token's bit for 32 bins
//     per word, which is what the all-bins scan consumes (the paper's own
//     layout in Section 4.2 keeps one token's bits of all bins contiguous
//     for the same reason).
//   bin-major (BM): bin x holds its 4^q-bit vector contiguously, which is
//     what a candidate check gathers.
//
// Each workgroup owns a tile of bins, builds the tile's bits in LDS with
// atomic ORs while walking the positions whose tokens can reach the tile,
// then writes the tile out with coalesced stores.

#include <algorithm>

#include "grim_internal.h"

namespace grim {
namespace {

__device__ __forceinline__ int base_code(uint32_t b) {
  const uint32_t u = b | 0x20u;
  if (u == 'a') return 0;
  if (u == 'c') return 1;
  if (u == 'g') return 2;
  if (u == 't') return 3;
  return -1;
}

constexpr int kRun = 32;  // consecutive token starts handled by one thread

// Walks token starts s in [lo, hi) in runs of kRun per thread and calls
// emit(code, s) for every valid token.
template <typename Emit>
__device__ __forceinline__ void for_tokens(const uint8_t* ref, uint64_t lo, uint64_t hi, uint32_t q,
                                           Emit emit) {
  const uint32_t qmask = (q >= 16) ? 0xFFFFFFFFu : ((1u << (2 * q)) - 1u);
  for (uint64_t s0 = lo + (uint64_t)threadIdx.x * kRun; s0 < hi; s0 += (uint64_t)blockDim.x * kRun) {
    const uint64_t s1 = s0 + kRun < hi ? s0 + kRun : hi;
    uint32_t code = 0, valid = 0;
    // prime with the first q-1 bases of the first window
    for (uint64_t p = s0; p + 1 < s0 + q; ++p) {
      const int b = base_code(ref[p]);
      valid = b < 0 ? 0 : valid + 1;
      code = ((code << 2) | (uint32_t)(b & 3)) & qmask;
    }
    for (uint64_t s = s0; s < s1; ++s) {
      const int b = base_code(ref[s + q - 1]);
      valid = b < 0 ? 0 : valid + 1;
      code = ((code << 2) | (uint32_t)(b & 3)) & qmask;
      if (valid >= q) emit(code, s);
    }
  }
}

// Bins whose extent holds token start s: [first_bin(s), s / B].
__device__ __forceinline__ uint64_t first_bin(uint64_t s, uint32_t B, uint32_t O) {
  const uint64_t ext = (uint64_t)B + O;
  return s < ext ? 0 : (s - ext) / B + 1;
}

template <int TW>
__global__ __launch_bounds__(1024) void k_build_tm(BuildArgs a) {
  constexpr int kMaxRows = TW == 32 ? 1024 : (TW == 8 ? 4096 : 16384);
  __shared__ uint32_t tile[kMaxRows * TW];
  const uint32_t R4 = 1u << (2 * a.q);
  const uint64_t w0 = (uint64_t)blockIdx.x * TW;          // first word of the tile
  const uint64_t x0 = w0 * 32;                             // first bin of the tile
  for (uint32_t i = threadIdx.x; i < R4 * TW; i += blockDim.x) tile[i] = 0;
  __syncthreads();
  if (x0 < a.nb) {
    const uint64_t xl = (x0 + 32ull * TW < a.nb ? x0 + 32ull * TW : a.nb) - 1;  // last bin
    const uint64_t last_start = a.G - a.q + 1;            // exclusive bound on starts
    uint64_t hi = xl * a.B + a.B + a.O;
    if (hi > last_start) hi = last_start;
    const uint64_t lo = x0 * a.B;
    if (lo < hi) {
      for_tokens(a.ref, lo, hi, a.q, [&](uint32_t code, uint64_t s) {
        uint64_t xa = first_bin(s, a.B, a.O);
        uint64_t xb = s / a.B;
        if (xa < x0) xa = x0;
        if (xb > xl) xb = xl;
        for (uint64_t x = xa; x <= xb; ++x) {
          const uint32_t lx = (uint32_t)(x - x0);
          atomicOr(&tile[code * TW + (lx >> 5)], 1u << (lx & 31));
        }
      });
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < R4 * TW; i += blockDim.x) {
    const uint32_t row = i / TW, w = i % TW;
    a.tm[(uint64_t)row * a.row_words + w0 + w] = tile[i];
  }
}

// Bin-major: a workgroup builds kBins consecutive bin vectors.
template <int VW>
__global__ __launch_bounds__(1024) void k_build_bm(BuildArgs a) {
  constexpr int kBins = VW >= 512 ? 16 : 32;
  __shared__ uint32_t vec[kBins * VW];
  const uint64_t x0 = (uint64_t)blockIdx.x * kBins;
  for (uint32_t i = threadIdx.x; i < kBins * VW; i += blockDim.x) vec[i] = 0;
  __syncthreads();
  const uint64_t xl = (x0 + kBins < a.nb ? x0 + kBins : a.nb) - 1;
  const uint64_t last_start = a.G - a.q + 1;
  uint64_t hi = xl * a.B + a.B + a.O;
  if (hi > last_start) hi = last_start;
  const uint64_t lo = x0 * a.B;
  if (lo < hi) {
    for_tokens(a.ref, lo, hi, a.q, [&](uint32_t code, uint64_t s) {
      uint64_t xa = first_bin(s, a.B, a.O);
      uint64_t xb = s / a.B;
      if (xa < x0) xa = x0;
      if (xb > xl) xb = xl;
      for (uint64_t x = xa; x <= xb; ++x)
        atomicOr(&vec[(uint32_t)(x - x0) * VW + (code >> 5)], 1u << (code & 31));
    });
  }
  __syncthreads();
  const uint64_t nbins = xl - x0 + 1;
  for (uint32_t i = threadIdx.x; i < nbins * VW; i += blockDim.x)
    a.bm[x0 * VW + i] = vec[i];
}

}  // namespace

hipError_t launch_build_tm(const BuildArgs& a, hipStream_t s) {
  const int TW = tm_tile_words(a.q);
  const uint64_t tiles = a.row_words / TW;
  if (tiles == 0) return hipSuccess;
  switch (TW) {
    case 32: hipLaunchKernelGGL(k_build_tm<32>, dim3((unsigned)tiles), dim3(1024), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_build_tm<8>, dim3((unsigned)tiles), dim3(1024), 0, s, a); break;
    default: hipLaunchKernelGGL(k_build_tm<2>, dim3((unsigned)tiles), dim3(1024), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_build_bm(const BuildArgs& a, hipStream_t s) {
  const uint32_t VW = a.vec_words;
  const int kBins = VW >= 512 ? 16 : 32;
  const uint64_t blocks = (a.nb + kBins - 1) / kBins;
  if (blocks == 0) return hipSuccess;
  switch (VW) {
    case 1: hipLaunchKernelGGL(k_build_bm<1>, dim3((unsigned)blocks), dim3(1024), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_build_bm<2>, dim3((unsigned)blocks), dim3(1024), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_build_bm<8>, dim3((unsigned)blocks), dim3(1024), 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_build_bm<32>, dim3((unsigned)blocks), dim3(1024), 0, s, a); break;
    case 128: hipLaunchKernelGGL(k_build_bm<128>, dim3((unsigned)blocks), dim3(1024), 0, s, a); break;
    case 512: hipLaunchKernelGGL(k_build_bm<512>, dim3((unsigned)blocks), dim3(1024), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Reference copy for verification: one base code per byte (grid-stride loop,
// the reference is read once, coalesced).
__global__ __launch_bounds__(256) void k_ref_codes(const uint8_t* ref, uint64_t G, uint8_t* codes) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < G; i += stride) {
    const uint8_t c = ref[i];
    uint8_t v = 4;
    switch (c | 0x20) {  // ASCII letters: fold to lower case
      case 'a': v = 0; break;
      case 'c': v = 1; break;
      case 'g': v = 2; break;
      case 't': v = 3; break;
      default: break;
    }
    codes[i] = v;
  }
}

hipError_t launch_ref_codes(const uint8_t* ref, uint64_t G, uint8_t* codes, hipStream_t s) {
  if (G == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((G + 255) / 256, 256ull * 64);
  hipLaunchKernelGGL(k_ref_codes, dim3((unsigned)blocks), dim3(256), 0, s, ref, G, codes);
  return hipGetLastError();
}

}  // namespace grim
