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

constexpr int kRun = 32;  // consecutive token starts handled by one thread

// Branch-free base code of one byte: with the case folded, d = byte - 0x60 is
// 1, 3, 7, 20 for a, c, g, t (bits of 0x10008A); ((d >> 1) ^ (d >> 2)) & 3
// maps those to 0, 1, 2, 3. *ok is false for any other byte.
__device__ __forceinline__ uint32_t base_code(uint32_t b, bool* ok) {
  const uint32_t d = (b | 0x20u) - 0x60u;
  *ok = d < 32u && ((0x0010008Au >> d) & 1u);
  return ((d >> 1) ^ (d >> 2)) & 3u;
}

// Walks the token starts s in [lo, hi) in runs of kRun consecutive starts per
// thread; runs begin at multiples of 16 bases so that a run's kRun + Q - 1
// bases come in with three 16-byte loads when the reference is 16-byte
// aligned (bases at or past G read as invalid). For every valid token it
// calls emit(code, x, rem) with x = s / B and rem = s % B, both tracked
// incrementally from one division per run.
template <int Q, typename Emit>
__device__ __forceinline__ void for_tokens(const uint8_t* ref, uint64_t G, bool aligned, uint64_t lo, uint64_t hi,
                                           uint32_t B, Emit emit) {
  constexpr int NB = kRun + Q - 1;       // bases a run spans
  constexpr int NV = (NB + 15) / 16;     // 16-byte loads
  constexpr uint32_t MASK = (Q >= 16) ? 0xFFFFFFFFu : ((1u << (2 * Q)) - 1u);
  const uint64_t base = lo & ~15ull;
  for (uint64_t s0 = base + (uint64_t)threadIdx.x * kRun; s0 < hi; s0 += (uint64_t)blockDim.x * kRun) {
    uint32_t w[NV * 4];
    if (aligned && s0 + NV * 16 <= G) {
      const uint4* src = reinterpret_cast<const uint4*>(ref + s0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const uint4 t = src[v];
        w[4 * v] = t.x; w[4 * v + 1] = t.y; w[4 * v + 2] = t.z; w[4 * v + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < NV * 4; ++k) {
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint64_t p = s0 + 4 * k + b;
          word |= (p < G ? (uint32_t)ref[p] : (uint32_t)'N') << (8 * b);
        }
        w[k] = word;
      }
    }
    uint64_t x = s0 / B;
    uint32_t rem = (uint32_t)(s0 - x * B);
    uint32_t code = 0;
    int run = 0;  // valid bases ending at the current one
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      bool ok;
      const uint32_t c = base_code((w[i >> 2] >> (8 * (i & 3))) & 0xFFu, &ok);
      run = ok ? run + 1 : 0;
      code = ((code << 2) | c) & MASK;
      if (i >= Q - 1) {
        const uint64_t s = s0 + (uint64_t)(i - (Q - 1));  // start of the window ending here
        if (run >= Q && s >= lo && s < hi) emit(code, x, rem);
        if (++rem == B) {
          rem = 0;
          ++x;
        }
      }
    }
  }
}

// Calls f(bin) for every bin in [x0, xl] whose extent [b*B, b*B + B + O)
// holds token start s = x*B + rem: bins x, x - 1, ... while rem + j*B < B + O.
template <typename F>
__device__ __forceinline__ void for_bins(uint64_t x, uint32_t rem, uint32_t B, uint32_t O, uint64_t x0, uint64_t xl,
                                         F f) {
  const uint64_t reach = (uint64_t)B + O;
  uint64_t off = rem;  // s - bin * B for bin = x - j
  for (uint64_t j = 0; j <= x && off < reach; ++j, off += B) {
    const uint64_t bin = x - j;
    if (bin < x0) break;
    if (bin <= xl) f(bin);
  }
}

// Token-major tile: TW words = 32 * TW bins, every row of R4 = 4^Q tokens, in LDS.
template <int Q>
__global__ __launch_bounds__(1024) void k_build_tm(BuildArgs a, bool aligned) {
  constexpr int TW = Q <= 5 ? 32 : (Q == 6 ? 8 : 2);
  constexpr uint32_t R4 = 1u << (2 * Q);
  __shared__ uint32_t tile[R4 * TW];
  const uint64_t w0 = (uint64_t)blockIdx.x * TW;  // first word of the tile
  const uint64_t x0 = w0 * 32;                     // first bin of the tile
  for (uint32_t i = threadIdx.x; i < R4 * TW; i += blockDim.x) tile[i] = 0;
  __syncthreads();
  if (x0 < a.nb) {
    const uint64_t xl = (x0 + 32ull * TW < a.nb ? x0 + 32ull * TW : a.nb) - 1;  // last bin
    const uint64_t last_start = a.G - Q + 1;                                     // exclusive bound on starts
    uint64_t hi = xl * a.B + a.B + a.O;
    if (hi > last_start) hi = last_start;
    const uint64_t lo = x0 * a.B;
    if (lo < hi) {
      for_tokens<Q>(a.ref, a.G, aligned, lo, hi, a.B, [&](uint32_t code, uint64_t x, uint32_t rem) {
        for_bins(x, rem, a.B, a.O, x0, xl, [&](uint64_t bin) {
          const uint32_t lx = (uint32_t)(bin - x0);
          atomicOr(&tile[code * TW + (lx >> 5)], 1u << (lx & 31));
        });
      });
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < R4 * TW; i += blockDim.x) {
    const uint32_t row = i / TW, w = i % TW;
    a.tm[(uint64_t)row * a.row_words + w0 + w] = tile[i];
  }
}

// Bin-major: a workgroup builds kBins consecutive bin vectors of VW words.
template <int Q>
__global__ __launch_bounds__(1024) void k_build_bm(BuildArgs a, bool aligned) {
  constexpr int VW = (1 << (2 * Q)) >= 32 ? (1 << (2 * Q)) / 32 : 1;
  constexpr int kBins = VW >= 512 ? 16 : 32;
  __shared__ uint32_t vec[kBins * VW];
  const uint64_t x0 = (uint64_t)blockIdx.x * kBins;
  for (uint32_t i = threadIdx.x; i < kBins * VW; i += blockDim.x) vec[i] = 0;
  __syncthreads();
  const uint64_t xl = (x0 + kBins < a.nb ? x0 + kBins : a.nb) - 1;
  const uint64_t last_start = a.G - Q + 1;
  uint64_t hi = xl * a.B + a.B + a.O;
  if (hi > last_start) hi = last_start;
  const uint64_t lo = x0 * a.B;
  if (lo < hi) {
    for_tokens<Q>(a.ref, a.G, aligned, lo, hi, a.B, [&](uint32_t code, uint64_t x, uint32_t rem) {
      for_bins(x, rem, a.B, a.O, x0, xl, [&](uint64_t bin) {
        atomicOr(&vec[(uint32_t)(bin - x0) * VW + (code >> 5)], 1u << (code & 31));
      });
    });
  }
  __syncthreads();
  const uint64_t nbins = xl - x0 + 1;
  for (uint32_t i = threadIdx.x; i < nbins * VW; i += blockDim.x) a.bm[x0 * VW + i] = vec[i];
}

}  // namespace

hipError_t launch_build_tm(const BuildArgs& a, hipStream_t s) {
  const int TW = tm_tile_words(a.q);
  const uint64_t tiles = a.row_words / TW;
  if (tiles == 0) return hipSuccess;
  const bool al = (reinterpret_cast<uintptr_t>(a.ref) & 15u) == 0;
  const dim3 g((unsigned)tiles), b(1024);
  switch (a.q) {
    case 1: hipLaunchKernelGGL(k_build_tm<1>, g, b, 0, s, a, al); break;
    case 2: hipLaunchKernelGGL(k_build_tm<2>, g, b, 0, s, a, al); break;
    case 3: hipLaunchKernelGGL(k_build_tm<3>, g, b, 0, s, a, al); break;
    case 4: hipLaunchKernelGGL(k_build_tm<4>, g, b, 0, s, a, al); break;
    case 5: hipLaunchKernelGGL(k_build_tm<5>, g, b, 0, s, a, al); break;
    case 6: hipLaunchKernelGGL(k_build_tm<6>, g, b, 0, s, a, al); break;
    case 7: hipLaunchKernelGGL(k_build_tm<7>, g, b, 0, s, a, al); break;
    default: return hipErrorInvalidValue;  // q = 8: a tile of 4^8 + 1 rows does not fit LDS
  }
  return hipGetLastError();
}

hipError_t launch_build_bm(const BuildArgs& a, hipStream_t s) {
  const uint32_t VW = a.vec_words;
  const int kBins = VW >= 512 ? 16 : 32;
  const uint64_t blocks = (a.nb + kBins - 1) / kBins;
  if (blocks == 0) return hipSuccess;
  const bool al = (reinterpret_cast<uintptr_t>(a.ref) & 15u) == 0;
  const dim3 g((unsigned)blocks), b(1024);
  switch (a.q) {
    case 1: hipLaunchKernelGGL(k_build_bm<1>, g, b, 0, s, a, al); break;
    case 2: hipLaunchKernelGGL(k_build_bm<2>, g, b, 0, s, a, al); break;
    case 3: hipLaunchKernelGGL(k_build_bm<3>, g, b, 0, s, a, al); break;
    case 4: hipLaunchKernelGGL(k_build_bm<4>, g, b, 0, s, a, al); break;
    case 5: hipLaunchKernelGGL(k_build_bm<5>, g, b, 0, s, a, al); break;
    case 6: hipLaunchKernelGGL(k_build_bm<6>, g, b, 0, s, a, al); break;
    case 7: hipLaunchKernelGGL(k_build_bm<7>, g, b, 0, s, a, al); break;
    case 8: hipLaunchKernelGGL(k_build_bm<8>, g, b, 0, s, a, al); break;
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
