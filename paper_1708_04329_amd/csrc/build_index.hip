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
// incrementally from one division per run (x < 2^31: at most 2^31 bins).
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
    // starts s0 + u with u in [u_lo, u_hi) lie in [lo, hi)
    const int u_lo = s0 < lo ? (int)(lo - s0) : 0;
    const int u_hi = hi - s0 < (uint64_t)kRun ? (int)(hi - s0) : kRun;
    const uint64_t x64 = s0 / B;
    uint32_t x = (uint32_t)x64;
    uint32_t rem = (uint32_t)(s0 - x64 * B);
    uint32_t code = 0;
    int run = 0;  // valid bases ending at the current one
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      bool ok;
      const uint32_t c = base_code((w[i >> 2] >> (8 * (i & 3))) & 0xFFu, &ok);
      run = ok ? run + 1 : 0;
      code = ((code << 2) | c) & MASK;
      if (i >= Q - 1) {
        const int u = i - (Q - 1);  // the window ending here starts at s0 + u
        if (run >= Q && u >= u_lo && u < u_hi) emit(code, x, rem);
        if (++rem == B) {
          rem = 0;
          ++x;
        }
      }
    }
  }
}

// Calls f(bin - x0) for every bin in [x0, xl] whose extent [b*B, b*B + B + O)
// holds token start s = x*B + rem: bins x, x - 1, ... while rem + j*B < B + O.
// When O <= B (every workload here) that is bin x, and bin x - 1 when rem < O:
// two predicated calls instead of a loop.
template <bool SHORT_O, typename F>
__device__ __forceinline__ void for_bins(uint32_t x, uint32_t rem, uint32_t B, uint32_t O, uint32_t x0, uint32_t xl,
                                         F f) {
  if constexpr (SHORT_O) {
    if (x >= x0 && x <= xl) f(x - x0);
    if (rem < O && x > x0 && x - 1 <= xl) f(x - 1 - x0);
    return;
  }
  const uint64_t reach = (uint64_t)B + O;
  uint64_t off = rem;  // s - bin * B for bin = x - j
  for (uint32_t bin = x;; --bin, off += B) {
    if (off >= reach || bin < x0) break;
    if (bin <= xl) f(bin - x0);
    if (bin == 0) break;
  }
}

// Words of a token-major row a build tile covers: 64 KB of LDS per tile (two
// workgroups of 1024 threads per CU), at most 32 words.
constexpr int build_tile_words(int q) { return q <= 4 ? 32 : (16384 >> (2 * q - 4)) / 16; }
static_assert(build_tile_words(5) == 16 && build_tile_words(6) == 4 && build_tile_words(7) == 1, "tile widths");

// Token-major tile: TW words = 32 * TW bins of every row of R4 = 4^Q tokens,
// in LDS word-major (word w of row t at w * R4 + (t ^ (w & SW))): the lanes of
// a wavefront take starts 32 bases apart, so most of them set bits of the same
// 32-bin word of random rows; with rows contiguous per word their atomics
// spread over the banks instead of all hitting one. The XOR keeps the
// row-major read-out (consecutive lanes: consecutive words of a row) off a
// single bank as well.
template <int Q, bool SHORT_O>
__global__ __launch_bounds__(1024) void k_build_tm(BuildArgs a, bool aligned) {
  constexpr int TW = build_tile_words(Q);
  constexpr uint32_t R4 = 1u << (2 * Q);
  constexpr uint32_t SW = (R4 < 32 ? R4 : 32) - 1;
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
      for_tokens<Q>(a.ref, a.G, aligned, lo, hi, a.B, [&](uint32_t code, uint32_t x, uint32_t rem) {
        for_bins<SHORT_O>(x, rem, a.B, a.O, (uint32_t)x0, (uint32_t)xl, [&](uint32_t lx) {
          const uint32_t w = lx >> 5;
          atomicOr(&tile[w * R4 + (code ^ (w & SW))], 1u << (lx & 31));
        });
      });
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < R4 * TW; i += blockDim.x) {
    const uint32_t row = i / TW, w = i % TW;
    a.tm[(uint64_t)row * a.row_words + w0 + w] = tile[w * R4 + (row ^ (w & SW))];
  }
}

// Bin-major: a workgroup builds kBins consecutive bin vectors of VW words.
template <int Q, bool SHORT_O>
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
    for_tokens<Q>(a.ref, a.G, aligned, lo, hi, a.B, [&](uint32_t code, uint32_t x, uint32_t rem) {
      for_bins<SHORT_O>(x, rem, a.B, a.O, (uint32_t)x0, (uint32_t)xl, [&](uint32_t lx) {
        atomicOr(&vec[lx * VW + (code >> 5)], 1u << (code & 31));
      });
    });
  }
  __syncthreads();
  const uint64_t nbins = xl - x0 + 1;
  for (uint32_t i = threadIdx.x; i < nbins * VW; i += blockDim.x) a.bm[x0 * VW + i] = vec[i];
}

template <int Q>
void launch_tm_q(const BuildArgs& a, bool al, dim3 g, hipStream_t s) {
  if (a.O <= a.B) hipLaunchKernelGGL((k_build_tm<Q, true>), g, dim3(1024), 0, s, a, al);
  else hipLaunchKernelGGL((k_build_tm<Q, false>), g, dim3(1024), 0, s, a, al);
}

template <int Q>
void launch_bm_q(const BuildArgs& a, bool al, dim3 g, hipStream_t s) {
  if (a.O <= a.B) hipLaunchKernelGGL((k_build_bm<Q, true>), g, dim3(1024), 0, s, a, al);
  else hipLaunchKernelGGL((k_build_bm<Q, false>), g, dim3(1024), 0, s, a, al);
}

}  // namespace

hipError_t launch_build_tm(const BuildArgs& a, hipStream_t s) {
  if (a.q < 1 || a.q > 7) return hipErrorInvalidValue;  // q = 8: a tile of 4^8 + 1 rows does not fit LDS
  const uint64_t tiles = a.row_words / build_tile_words((int)a.q);
  if (tiles == 0) return hipSuccess;
  const bool al = (reinterpret_cast<uintptr_t>(a.ref) & 15u) == 0;
  const dim3 g((unsigned)tiles);
  switch (a.q) {
    case 1: launch_tm_q<1>(a, al, g, s); break;
    case 2: launch_tm_q<2>(a, al, g, s); break;
    case 3: launch_tm_q<3>(a, al, g, s); break;
    case 4: launch_tm_q<4>(a, al, g, s); break;
    case 5: launch_tm_q<5>(a, al, g, s); break;
    case 6: launch_tm_q<6>(a, al, g, s); break;
    default: launch_tm_q<7>(a, al, g, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_build_bm(const BuildArgs& a, hipStream_t s) {
  const uint32_t VW = a.vec_words;
  const int kBins = VW >= 512 ? 16 : 32;
  const uint64_t blocks = (a.nb + kBins - 1) / kBins;
  if (blocks == 0) return hipSuccess;
  const bool al = (reinterpret_cast<uintptr_t>(a.ref) & 15u) == 0;
  const dim3 g((unsigned)blocks);
  switch (a.q) {
    case 1: launch_bm_q<1>(a, al, g, s); break;
    case 2: launch_bm_q<2>(a, al, g, s); break;
    case 3: launch_bm_q<3>(a, al, g, s); break;
    case 4: launch_bm_q<4>(a, al, g, s); break;
    case 5: launch_bm_q<5>(a, al, g, s); break;
    case 6: launch_bm_q<6>(a, al, g, s); break;
    case 7: launch_bm_q<7>(a, al, g, s); break;
    case 8: launch_bm_q<8>(a, al, g, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Reference copy for verification: one base code per byte (0..3 for A, C, G,
// T in either case, 4 for any other byte).
//
// Four bytes at once: with the case folded (l = b | 0x20), bits 1-2 and 2-3 of
// a, c, g, t (0x61, 0x63, 0x67, 0x74) XOR to their codes 0, 1, 2, 3; a byte is
// a base exactly when it equals the letter its code names, which one byte
// permute looks up, and bytes that differ take code 4.
__device__ __forceinline__ uint32_t ref_codes4(uint32_t w) {
  const uint32_t l = w | 0x20202020u;
  const uint32_t c = ((l >> 1) ^ (l >> 2)) & 0x03030303u;
  const uint32_t letter = __builtin_amdgcn_perm(0u, 0x74676361u, c);  // byte k = "acgt"[c_k]
  const uint32_t d = letter ^ l;
  // 1 in each byte of d that is not zero (the add stays within the byte)
  const uint32_t bad = ((((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u) >> 7;
  return (c & ~(bad * 3u)) | (bad << 2);
}

// 16 bytes per lane when both pointers are 16-byte aligned (the copy is one
// read and one write of G bytes); the last G % 16 bytes, or all of them for an
// unaligned reference, go one byte per lane with the same arithmetic.
__global__ __launch_bounds__(256) void k_ref_codes(const uint8_t* ref, uint64_t G, uint8_t* codes, bool vec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n16 = vec ? G / 16 : 0;
  const uint4* src = reinterpret_cast<const uint4*>(ref);
  uint4* dst = reinterpret_cast<uint4*>(codes);
  for (uint64_t i = tid; i < n16; i += stride) {
    const uint4 t = src[i];
    dst[i] = make_uint4(ref_codes4(t.x), ref_codes4(t.y), ref_codes4(t.z), ref_codes4(t.w));
  }
  for (uint64_t i = n16 * 16 + tid; i < G; i += stride) codes[i] = (uint8_t)ref_codes4(ref[i]);
}

hipError_t launch_ref_codes(const uint8_t* ref, uint64_t G, uint8_t* codes, hipStream_t s) {
  if (G == 0) return hipSuccess;
  const bool vec = ((reinterpret_cast<uintptr_t>(ref) | reinterpret_cast<uintptr_t>(codes)) & 15u) == 0;
  const uint64_t items = vec ? G / 16 + 16 : G;
  const uint64_t blocks = std::min<uint64_t>((items + 255) / 256, 256ull * 8);
  hipLaunchKernelGGL(k_ref_codes, dim3((unsigned)blocks), dim3(256), 0, s, ref, G, codes, vec);
  return hipGetLastError();
}

}  // namespace grim
