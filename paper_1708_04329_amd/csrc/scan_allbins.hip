// All-bins filter: accumulate + threshold (paper Section 3 steps 2-3 for
// every bin, Section 4.2 "one sum and one comparator per bin").
//
// For read r and bin x the filter needs count[r][x] = sum over the read's
// token positions i of bit[x][t_{r,i}], and pass = count >= T_r. With the
// token-major index, the bits of one token for 32 consecutive bins form one
// uint32 word, so a word-wide adder advances 32 bin counters at once. The
// counters are kept bit-sliced: plane k holds bit k of 32 counters. Tokens
// are folded in with a carry-save (Harley-Seal) tree of full adders; on gfx950
// a full adder is two v_bitop3_b32 instructions (xor3 for the sum, majority
// for the carry), so each token costs about two VALU operations per 32 bins.
// The threshold test adds K = 2^P - T_r to the P-plane counters and keeps the
// carry out of the top plane (count >= T_r exactly when that carry is 1): one
// majority per plane.
//
// Work split: a workgroup owns one tile of TW words (32*TW bins) and a chunk
// of reads. It copies the tile's 4^q rows (plus an all-zero row for invalid
// and padding tokens) from HBM into LDS once, then every read of the chunk
// streams its token list against the LDS rows: G = TW/LW lanes share a read,
// each lane owns LW words (32*LW bins) and reads them with LW/4 16-byte LDS
// loads per token. Tokens arrive pre-scaled to the LDS byte offset of their
// row, so a row address costs one add per token. Workgroup ids are remapped
// so the 32 CUs of one XCD work on the tiles of the same read chunk, whose
// tokens then stay in that XCD's L2.

#include "grim_internal.h"

namespace grim {
namespace {

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// Full adder on 32 lanes of bits: (carry, sum) of a + b + c. Both functions
// are symmetric in their inputs, so the operand order of bitop3 is immaterial.
#define CSA(carry, sum, a, b, c)              \
  do {                                        \
    const uint32_t _a = (a), _b = (b), _c = (c); \
    carry = maj3(_a, _b, _c);                 \
    sum = xor3(_a, _b, _c);                   \
  } while (0)

template <int LW>
struct Words {
  uint32_t w[LW];
};

template <int LW>
__device__ __forceinline__ Words<LW> lds_row(const uint32_t* p) {
  Words<LW> r;
  if constexpr (LW == 8) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const uint4 u = *reinterpret_cast<const uint4*>(p + 4);
    r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
    r.w[4] = u.x; r.w[5] = u.y; r.w[6] = u.z; r.w[7] = u.w;
  } else if constexpr (LW == 4) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
  } else if constexpr (LW == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    r.w[0] = v.x; r.w[1] = v.y;
  } else {
    r.w[0] = p[0];
  }
  return r;
}

// Bit-sliced counters of LW words: planes 0..4 are the Harley-Seal level
// accumulators (ones, twos, fours, eights, sixteens), planes 5.. hold the
// multiples of 32 in binary.
template <int LW, int NHI>
struct Counters {
  uint32_t p[5 + NHI][LW];
};

// Fold 32 tokens (tk[i] = LDS byte offset of token i's row) into the counters.
template <int LW, int NHI>
__device__ __forceinline__ void fold32(Counters<LW, NHI>& c, const char* lds_lane, const uint32_t (&tk)[32]) {
  auto row = [&](int i) -> Words<LW> {
    return lds_row<LW>(reinterpret_cast<const uint32_t*>(lds_lane + tk[i]));
  };
  uint32_t s16a[LW], s16b[LW];
#pragma unroll
  for (int h16 = 0; h16 < 2; ++h16) {
    uint32_t e8a[LW], e8b[LW];
#pragma unroll
    for (int h8 = 0; h8 < 2; ++h8) {
      uint32_t f4a[LW], f4b[LW];
#pragma unroll
      for (int h4 = 0; h4 < 2; ++h4) {
        const int i0 = h16 * 16 + h8 * 8 + h4 * 4;
        const Words<LW> x0 = row(i0), x1 = row(i0 + 1), x2 = row(i0 + 2), x3 = row(i0 + 3);
        uint32_t t2a[LW], t2b[LW];
#pragma unroll
        for (int j = 0; j < LW; ++j) {
          CSA(t2a[j], c.p[0][j], c.p[0][j], x0.w[j], x1.w[j]);
          CSA(t2b[j], c.p[0][j], c.p[0][j], x2.w[j], x3.w[j]);
          if (h4 == 0) CSA(f4a[j], c.p[1][j], c.p[1][j], t2a[j], t2b[j]);
          else CSA(f4b[j], c.p[1][j], c.p[1][j], t2a[j], t2b[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < LW; ++j) {
        if (h8 == 0) CSA(e8a[j], c.p[2][j], c.p[2][j], f4a[j], f4b[j]);
        else CSA(e8b[j], c.p[2][j], c.p[2][j], f4a[j], f4b[j]);
      }
      // keep the scheduler from hoisting the next 8 tokens' LDS loads above
      // this point: with 8 words per lane, 32 tokens of loads in flight would
      // not fit the register file
      if constexpr (LW >= 8) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < LW; ++j) {
      if (h16 == 0) CSA(s16a[j], c.p[3][j], c.p[3][j], e8a[j], e8b[j]);
      else CSA(s16b[j], c.p[3][j], c.p[3][j], e8a[j], e8b[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < LW; ++j) {
    uint32_t carry;
    CSA(carry, c.p[4][j], c.p[4][j], s16a[j], s16b[j]);
    // ripple the multiple of 32 into the high planes
#pragma unroll
    for (int k = 0; k < NHI; ++k) {
      const uint32_t h = c.p[5 + k][j];
      c.p[5 + k][j] = h ^ carry;
      if (k + 1 < NHI) carry = h & carry;
    }
  }
}

// Threshold test on 32 bit-sliced counters of NP planes: bit b of the result
// is (counter_b >= T). With K = 2^NP - T the counter reaches T exactly when
// counter + K carries out of plane NP-1; the carry chain is one majority per
// plane (km[k] = all-ones when bit k of K is set). T <= 0 passes every bin.
template <int NP>
__device__ __forceinline__ uint32_t ge_threshold(const uint32_t (&pl)[NP], const uint32_t (&km)[NP],
                                                 uint32_t allpass) {
  uint32_t carry = pl[0] & km[0];
#pragma unroll
  for (int k = 1; k < NP; ++k) carry = maj3(pl[k], km[k], carry);
  return carry | allpass;
}

template <int LW, int NHI>
__device__ __forceinline__ void scan_read(const ScanArgs& a, const char* lds_lane, bool active,
                                          const uint32_t* tok, uint32_t* out_row, uint64_t rid, uint32_t ntok,
                                          int32_t T, uint64_t gw0) {
  constexpr int NP = 5 + NHI;
  Counters<LW, NHI> c;
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int j = 0; j < LW; ++j) c.p[k][j] = 0;
  const uint32_t nblk = active ? (ntok + 31) >> 5 : 0;
  const uint4* tk4 = reinterpret_cast<const uint4*>(tok);
  for (uint32_t b = 0; b < nblk; ++b) {
    uint32_t tk[32];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint4 v = tk4[b * 8 + i];
      tk[4 * i + 0] = v.x; tk[4 * i + 1] = v.y; tk[4 * i + 2] = v.z; tk[4 * i + 3] = v.w;
    }
    fold32<LW, NHI>(c, lds_lane, tk);
  }
  if (!active) return;
  // K = 2^NP - T as NP all-ones/all-zeros masks, shared by the lane's words
  const uint32_t allpass = T <= 0 ? 0xFFFFFFFFu : 0u;
  const uint32_t K = T <= 0 ? 0u : (uint32_t)((1u << NP) - (uint32_t)T);
  uint32_t km[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) km[k] = ((K >> k) & 1u) ? 0xFFFFFFFFu : 0u;
#pragma unroll
  for (int j = 0; j < LW; ++j) {
    const uint64_t gw = gw0 + j;
    if (gw >= a.W) continue;
    uint32_t pl[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) pl[k] = c.p[k][j];
    uint32_t ge = ge_threshold<NP>(pl, km, allpass);
    if (gw == a.W - 1 && (a.nb & 31)) ge &= (1u << (a.nb & 31)) - 1u;
    out_row[gw] = ge;
    if (a.counts_out) {
      const uint64_t xb = gw * 32;
      for (int b = 0; b < 32; ++b) {
        if (xb + b >= a.nb) break;
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) v |= ((pl[k] >> b) & 1u) << k;
        if (a.counts_bytes == 1) reinterpret_cast<uint8_t*>(a.counts_out)[rid * a.nb + xb + b] = (uint8_t)v;
        else reinterpret_cast<uint16_t*>(a.counts_out)[rid * a.nb + xb + b] = (uint16_t)v;
      }
    }
  }
}

template <int TW, int LW, int NT>
__global__ __launch_bounds__(NT) void k_scan_allbins(ScanArgs a) {
  constexpr int G = TW / LW;       // lanes per read
  constexpr int RPW = 64 / G;      // reads per wavefront
  constexpr int NW = NT / 64;
  constexpr int kMaxRows = TW == 32 ? 1024 : (TW == 8 ? 4096 : 16384);
  __shared__ __attribute__((aligned(16))) uint32_t lds[(kMaxRows + 1) * TW];

  // workgroup -> (read chunk, tile), XCD-aware: ids i and i+8 share an XCD
  const uint32_t id = blockIdx.x;
  const uint32_t xcd = id & 7u, slot = id >> 3;
  const uint32_t rc_local = slot / a.n_tiles;
  const uint32_t tile = slot - rc_local * a.n_tiles;
  const uint32_t rchunk = rc_local * 8u + xcd;
  if (rchunk >= a.n_rchunks) return;
  const uint64_t n_reads = a.dyn ? min(a.dyn->n_reads, a.n_reads) : a.n_reads;
  if ((uint64_t)rchunk * a.reads_per_chunk >= n_reads) return;
  if (a.status && a.status[0] != 0) return;  // inputs were rejected: leave outputs untouched

  // stage the tile: rows 0..R4-1 from HBM, row R4 = zeros
  const uint32_t R4 = a.R4;
  constexpr int V4 = TW / 4 > 0 ? TW / 4 : 1;
  if constexpr (TW >= 4) {
    const uint4* src = reinterpret_cast<const uint4*>(a.tm);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    const uint64_t row4 = a.row_words / 4;
    const uint64_t col4 = (uint64_t)tile * TW / 4;
    for (uint32_t i = threadIdx.x; i < R4 * V4; i += NT) {
      const uint32_t row = i / V4, c = i % V4;
      dst[i] = src[row * row4 + col4 + c];
    }
  } else {
    for (uint32_t i = threadIdx.x; i < R4 * TW; i += NT) {
      const uint32_t row = i / TW, c = i % TW;
      lds[i] = a.tm[(uint64_t)row * a.row_words + (uint64_t)tile * TW + c];
    }
  }
  for (uint32_t i = threadIdx.x; i < TW; i += NT) lds[R4 * TW + i] = 0;
  __syncthreads();

  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t g = lane / G, s = lane % G;
  const char* lds_lane = reinterpret_cast<const char*>(lds) + s * LW * 4;
  const uint64_t gw0 = (uint64_t)tile * TW + (uint64_t)s * LW;
  const uint64_t r_begin = (uint64_t)rchunk * a.reads_per_chunk;
  uint64_t r_end = r_begin + a.reads_per_chunk;
  if (r_end > n_reads) r_end = n_reads;

  for (uint64_t base = r_begin + (uint64_t)wave * RPW; base < r_end; base += (uint64_t)NW * RPW) {
    const uint64_t k = base + g;
    const bool active = k < r_end;
    uint64_t rid = 0;
    const uint32_t* tok = nullptr;
    uint32_t* out_row = nullptr;
    uint32_t ntok = 0;
    int32_t T = 0;
    if (active) {
      rid = a.read_order ? a.read_order[k] : k;
      if (a.desc) {
        const ReadDesc d = a.desc[rid];
        tok = d.tok;
        out_row = d.out;
        ntok = d.ntok;
        T = d.T;
      } else {
        const int64_t o0 = a.offsets[rid], o1 = a.offsets[rid + 1];
        ntok = (uint32_t)(o1 - o0 - a.q + 1);
        tok = a.tokens + token_base(o0, rid);
        out_row = a.mask_out + rid * a.W;
        T = a.thr[rid];
      }
    }
    if (__any(ntok > 255)) scan_read<LW, 11>(a, lds_lane, active, tok, out_row, rid, ntok, T, gw0);
    else scan_read<LW, 3>(a, lds_lane, active, tok, out_row, rid, ntok, T, gw0);
  }
}

template <int TW, int LW, int NT>
hipError_t launch_t(const ScanArgs& a, hipStream_t s) {
  const uint64_t per_xcd = (a.n_rchunks + 7) / 8;
  const uint64_t blocks = 8ull * per_xcd * a.n_tiles;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_scan_allbins<TW, LW, NT>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_allbins(const ScanArgs& a0, const ScanConfig& cfg, hipStream_t s) {
  ScanArgs a = a0;
  const int TW = tm_tile_words(a.q);
  a.reads_per_chunk = (uint32_t)cfg.reads_per_chunk;
  a.n_tiles = (uint32_t)((a.W + TW - 1) / TW);
  a.n_rchunks = (uint32_t)((a.n_reads + a.reads_per_chunk - 1) / a.reads_per_chunk);
  if (a.n_reads == 0 || a.n_tiles == 0) return hipSuccess;
  const int nt = cfg.threads;
  const bool w8 = cfg.lane_words == 8;
#define GRIM_SCAN_NT(TW_, LW_)                                              \
  do {                                                                      \
    if (nt == 1024) return launch_t<TW_, LW_, 1024>(a, s);                  \
    if (nt == 256) return launch_t<TW_, LW_, 256>(a, s);                    \
    return launch_t<TW_, LW_, 512>(a, s);                                   \
  } while (0)
  switch (TW) {
    case 32:
      if (w8) GRIM_SCAN_NT(32, 8);
      GRIM_SCAN_NT(32, 4);
    case 8:
      if (w8) GRIM_SCAN_NT(8, 8);
      GRIM_SCAN_NT(8, 4);
    default:
      GRIM_SCAN_NT(2, 2);
  }
#undef GRIM_SCAN_NT
}

}  // namespace grim
