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
// tokens then stay in that XCD's L2; chunks go round-robin to the XCDs, and
// their number is a multiple of 8, so each XCD gets the same work.
//
// Full 32-token blocks go through the Harley-Seal tree, two blocks per step
// so that only every other block's carry ripples through the upper planes;
// their tokens and rows are loaded ahead of use through register rings.
// Each read's tokens arrive ordered by the parity of their row (see the
// tokenizer and the length order), so the two reads that share a bank pass
// of an LDS read take rows in opposite halves of the banks.
// The remainder of a read is folded first, exactly, as power-of-two parts in
// increasing size: each part's carry lands in a still-empty plane and needs
// no ripple, and no padding token costs work unless another read of the
// wavefront needs that part. Counters have
// 8 planes (counts up to 255); a wavefront holding a longer read switches to
// 16 planes and covers its words in 2-word passes, which keeps that path
// within the registers of the common one.

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

// Add a carry of weight 2^L (one bit per bin) to the counters: half adders up
// through planes L..4, then the binary planes of weight 32 and up.
template <int L, int LW, int NHI>
__device__ __forceinline__ void add_carry(Counters<LW, NHI>& c, const uint32_t (&carry_in)[LW]) {
#pragma unroll
  for (int j = 0; j < LW; ++j) {
    uint32_t carry = carry_in[j];
#pragma unroll
    for (int k = L; k < 5 + NHI; ++k) {
      const uint32_t h = c.p[k][j];
      c.p[k][j] = h ^ carry;
      if (k + 1 < 5 + NHI) carry = h & carry;
    }
  }
}

// The 32 token offsets of one full block.
__device__ __forceinline__ void load_block(uint32_t (&tk)[32], const uint32_t* src) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint4 v = ldg4(src + 4 * i);
    tk[4 * i + 0] = v.x; tk[4 * i + 1] = v.y; tk[4 * i + 2] = v.z; tk[4 * i + 3] = v.w;
  }
}

// Full blocks stream through two rings held in registers. A stretch of 64
// tokens (two blocks) is folded per loop iteration; chunk j (tokens 4j..4j+3)
// of the stretch sits in token slot j % 4 and is loaded from global memory
// three chunks before it is needed, and token i's row sits in row slot i % 4
// and is read from LDS four tokens before it is needed. Both rings wrap at 64
// tokens, so the slots line up from one stretch to the next: the last steps
// of a stretch already load the next stretch's first chunks and rows. Each
// step ends at a scheduling barrier, which keeps the loads where they are
// written: two pairs of LDS reads and up to three token chunks stay in flight
// while a pair of rows is folded, instead of a wait on every pair.
template <int LW>
struct Ring {
  uint32_t tq[4][4];
  Words<LW> rq[4];
};

// Load token chunk J of the stretch at `src` (the stretch's first token).
template <int J, int LW>
__device__ __forceinline__ void ring_chunk(Ring<LW>& R, const uint32_t* src) {
  const uint4 v = ldg4(src + 4 * J);
  R.tq[J % 4][0] = v.x; R.tq[J % 4][1] = v.y; R.tq[J % 4][2] = v.z; R.tq[J % 4][3] = v.w;
}

// Read token I's row from LDS into its slot.
template <int I, int LW>
__device__ __forceinline__ void ring_row(Ring<LW>& R, const char* lds_lane) {
  R.rq[I % 4] = lds_row<LW>(reinterpret_cast<const uint32_t*>(lds_lane + R.tq[(I / 4) % 4][I % 4]));
}

// tree<N> over tokens I .. I+N-1 of the stretch, rows taken from the ring.
template <int N, int I, int LW, int NHI>
__device__ __forceinline__ void ring_tree(Counters<LW, NHI>& c, Ring<LW>& R, const char* lds_lane,
                                          const uint32_t* src, uint32_t (&out)[LW]) {
  if constexpr (N == 2) {
    if constexpr (I % 4 == 0) ring_chunk<I / 4 + 3, LW>(R, src);
    const Words<LW> x0 = R.rq[I % 4], x1 = R.rq[(I + 1) % 4];
#pragma unroll
    for (int j = 0; j < LW; ++j) CSA(out[j], c.p[0][j], c.p[0][j], x0.w[j], x1.w[j]);
    __builtin_amdgcn_sched_barrier(0);
    ring_row<I + 4, LW>(R, lds_lane);
    ring_row<I + 5, LW>(R, lds_lane);
    __builtin_amdgcn_sched_barrier(0);
  } else {
    constexpr int L = (N == 4) ? 1 : (N == 8) ? 2 : (N == 16) ? 3 : 4;
    uint32_t a[LW], b[LW];
    ring_tree<N / 2, I, LW, NHI>(c, R, lds_lane, src, a);
    ring_tree<N / 2, I + N / 2, LW, NHI>(c, R, lds_lane, src, b);
#pragma unroll
    for (int j = 0; j < LW; ++j) CSA(out[j], c.p[L][j], c.p[L][j], a[j], b[j]);
  }
}

// Load N = 2^k token offsets from global memory at `src` (16-byte aligned
// for N >= 4).
template <int N>
__device__ __forceinline__ void load_part(uint32_t (&tk)[N], const uint32_t* src) {
  if constexpr (N >= 4) {
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const uint4 v = ldg4(src + 4 * i);
      tk[4 * i + 0] = v.x; tk[4 * i + 1] = v.y; tk[4 * i + 2] = v.z; tk[4 * i + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) tk[i] = ldg1(src + i);
  }
}

// The remainder parts and an odd full block take their tokens from registers
// (loaded together before the first fold) and their rows through a ring of
// four, read from LDS four tokens ahead, as in the block loop.
template <int LW>
struct Rows {
  Words<LW> rq[4];
};

template <int I, int N, int LW>
__device__ __forceinline__ void part_row(Rows<LW>& R, const char* lds_lane, const uint32_t* tk) {
  if constexpr (I < N) R.rq[I % 4] = lds_row<LW>(reinterpret_cast<const uint32_t*>(lds_lane + tk[I]));
}

// tree<M> over tokens I .. I+M-1 of an N-token part, rows from the ring.
template <int M, int I, int N, int LW, int NHI>
__device__ __forceinline__ void part_tree(Counters<LW, NHI>& c, Rows<LW>& R, const char* lds_lane, const uint32_t* tk,
                                          uint32_t (&out)[LW]) {
  if constexpr (M == 2) {
    const Words<LW> x0 = R.rq[I % 4], x1 = R.rq[(I + 1) % 4];
#pragma unroll
    for (int j = 0; j < LW; ++j) CSA(out[j], c.p[0][j], c.p[0][j], x0.w[j], x1.w[j]);
    __builtin_amdgcn_sched_barrier(0);
    part_row<I + 4, N, LW>(R, lds_lane, tk);
    part_row<I + 5, N, LW>(R, lds_lane, tk);
    __builtin_amdgcn_sched_barrier(0);
  } else {
    constexpr int L = (M == 4) ? 1 : (M == 8) ? 2 : (M == 16) ? 3 : 4;
    uint32_t a[LW], b[LW];
    part_tree<M / 2, I, N, LW, NHI>(c, R, lds_lane, tk, a);
    part_tree<M / 2, I + M / 2, N, LW, NHI>(c, R, lds_lane, tk, b);
#pragma unroll
    for (int j = 0; j < LW; ++j) CSA(out[j], c.p[L][j], c.p[L][j], a[j], b[j]);
  }
}

// Fold N = 2^k tokens into the counters, whose planes k and up are still
// zero; the tree's carry of weight 2^k becomes plane k.
template <int N, int LW, int NHI>
__device__ __forceinline__ void fold_into_empty(Counters<LW, NHI>& c, const char* lds_lane, const uint32_t (&tk)[N]) {
  constexpr int L = (N == 1) ? 0 : (N == 2) ? 1 : (N == 4) ? 2 : (N == 8) ? 3 : (N == 16) ? 4 : 5;
  if constexpr (N == 1) {
    const Words<LW> x = lds_row<LW>(reinterpret_cast<const uint32_t*>(lds_lane + tk[0]));
#pragma unroll
    for (int j = 0; j < LW; ++j) c.p[0][j] = x.w[j];
  } else {
    Rows<LW> R;
    part_row<0, N, LW>(R, lds_lane, tk);
    part_row<1, N, LW>(R, lds_lane, tk);
    part_row<2, N, LW>(R, lds_lane, tk);
    part_row<3, N, LW>(R, lds_lane, tk);
    uint32_t carry[LW];
    part_tree<N, 0, N, LW, NHI>(c, R, lds_lane, tk, carry);
#pragma unroll
    for (int j = 0; j < LW; ++j) c.p[L][j] = carry[j];
  }
}

// Threshold test on 32 bit-sliced counters of NP planes: bit b of the result
// is (counter_b >= T). With K = 2^NP - T the counter reaches T exactly when
// counter + K carries out of plane NP-1; the carry chain is one majority per
// plane (km[k] = all-ones when bit k of K is set). T <= 0 passes every bin:
// then K = 2^NP - 1 with a carry into plane 0 (cin all-ones), so the sum
// always reaches 2^NP.
template <int NP>
__device__ __forceinline__ uint32_t ge_threshold(const uint32_t (&pl)[NP], const uint32_t (&km)[NP], uint32_t cin) {
  uint32_t carry = cin;
#pragma unroll
  for (int k = 0; k < NP; ++k) carry = maj3(pl[k], km[k], carry);
  return carry;
}

template <int LW, int NHI, bool COUNTS>
__device__ __forceinline__ void scan_read(const ScanArgs& a, const char* lds_lane, bool active,
                                          const uint32_t* tok, uint32_t* out_row, uint64_t rid, uint32_t ntok,
                                          int32_t T, uint64_t gw0) {
  constexpr int NP = 5 + NHI;
  Counters<LW, NHI> c;
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int j = 0; j < LW; ++j) c.p[k][j] = 0;
  // A lane without a read of its own (ntok = 0) streams the tokens of another
  // read of its chunk and stores nothing, so no load needs a guard.
  const uint32_t nfull = ntok >> 5;
  // The last partial block first, folded exactly as 1/2/4/8/16-token parts
  // into the empty counters: part 2^k is folded when any lane's remainder
  // has bit k, so the parts cover every lane's remainder, and a lane reads
  // zero-row padding past its own (every token list ends with at least one
  // padding token and is padded to a multiple of 32). The parts' token loads
  // are all issued before the first fold so that their latencies overlap.
  const uint32_t rem = ntok & 31u;
  const uint32_t* tail = tok + nfull * 32;
  const bool h16 = __any(rem & 16u), h8 = __any(rem & 8u), h4 = __any(rem & 4u), h2 = __any(rem & 2u),
             h1 = __any(rem & 1u);
  const uint32_t p8 = h16 ? 16 : 0, p4 = p8 + (h8 ? 8 : 0), p2 = p4 + (h4 ? 4 : 0), p1 = p2 + (h2 ? 2 : 0);
  uint32_t t16[16], t8[8], t4[4], t2[2], t1[1];
  if (h16) load_part<16>(t16, tail);
  if (h8) load_part<8>(t8, tail + p8);
  if (h4) load_part<4>(t4, tail + p4);
  if (h2) load_part<2>(t2, tail + p2);
  if (h1) load_part<1>(t1, tail + p1);
  if (h1) fold_into_empty<1, LW, NHI>(c, lds_lane, t1);
  if (h2) fold_into_empty<2, LW, NHI>(c, lds_lane, t2);
  if (h4) fold_into_empty<4, LW, NHI>(c, lds_lane, t4);
  if (h8) fold_into_empty<8, LW, NHI>(c, lds_lane, t8);
  if (h16) fold_into_empty<16, LW, NHI>(c, lds_lane, t16);
  // An odd full block goes next, as a part of 32: the count is still below 32,
  // so its weight-32 carry becomes plane 5. Then the remaining full blocks,
  // two at a time: the weight-32 carries of the two trees meet in one full
  // adder at plane 5, and only its carry ripples on.
  uint32_t b = 0;
  if (nfull & 1u) {
    uint32_t tk[32];
    load_block(tk, tok);
    fold_into_empty<32, LW, NHI>(c, lds_lane, tk);
    b = 1;
  }
  if (b + 2 <= nfull) {
    Ring<LW> R;
    const uint32_t* src = tok + b * 32;
    ring_chunk<0, LW>(R, src);
    ring_chunk<1, LW>(R, src);
    ring_chunk<2, LW>(R, src);
    ring_row<0, LW>(R, lds_lane);
    ring_row<1, LW>(R, lds_lane);
    ring_row<2, LW>(R, lds_lane);
    ring_row<3, LW>(R, lds_lane);
    for (; b + 2 <= nfull; b += 2, src += 64) {
      uint32_t c1[LW], c2[LW], c64[LW];
      ring_tree<32, 0, LW, NHI>(c, R, lds_lane, src, c1);
      ring_tree<32, 32, LW, NHI>(c, R, lds_lane, src, c2);
#pragma unroll
      for (int j = 0; j < LW; ++j) CSA(c64[j], c.p[5][j], c.p[5][j], c1[j], c2[j]);
      add_carry<6, LW, NHI>(c, c64);
    }
  }
  if (!active) return;
  // K = 2^NP - T as NP all-ones/all-zeros masks, shared by the lane's words
  const uint32_t cin = T <= 0 ? 0xFFFFFFFFu : 0u;
  const uint32_t K = T <= 0 ? (1u << NP) - 1u : (uint32_t)((1u << NP) - (uint32_t)T);
  uint32_t km[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) km[k] = ((K >> k) & 1u) ? 0xFFFFFFFFu : 0u;
  if (!COUNTS && gw0 + LW < a.W) {
    // every word of the lane is a whole word of the row: no range or tail checks
    uint32_t* o = out_row + gw0;
#pragma unroll
    for (int j = 0; j < LW; ++j) {
      uint32_t pl[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) pl[k] = c.p[k][j];
      o[j] = ge_threshold<NP>(pl, km, cin);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < LW; ++j) {
    const uint64_t gw = gw0 + j;
    if (gw >= a.W) continue;
    uint32_t pl[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) pl[k] = c.p[k][j];
    uint32_t ge = ge_threshold<NP>(pl, km, cin);
    if (gw == a.W - 1 && (a.nb & 31)) ge &= (1u << (a.nb & 31)) - 1u;
    out_row[gw] = ge;
    if (COUNTS && a.counts_out) {
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

template <int TW, int LW, int NT, bool COUNTS>
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
  // The reads' workgroup iterations are dealt out evenly over the chunks
  // (sizes differ by at most one iteration); with a chunk count that is a
  // multiple of 8, every XCD gets the same share of the work.
  constexpr uint32_t kIter = (uint32_t)(NW * RPW);
  const uint64_t n_iter = (n_reads + kIter - 1) / kIter;
  const uint64_t per = n_iter / a.n_rchunks, extra = n_iter % a.n_rchunks;
  const uint64_t it0 = (uint64_t)rchunk * per + min((uint64_t)rchunk, extra);
  const uint64_t its = per + (rchunk < extra ? 1 : 0);
  const uint64_t r_begin = it0 * kIter;
  uint64_t r_end = r_begin + its * kIter;
  if (r_end > n_reads) r_end = n_reads;
  if (r_begin >= r_end) return;
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
  // groups of RPW reads go to the wavefronts in order of demand: each takes
  // group `wave` first, then the next unclaimed one, so the workgroup ends
  // when its last group ends rather than with its slowest wavefront's share
  __shared__ uint32_t next_group;
  if (threadIdx.x == 0) next_group = NW;
  __syncthreads();

  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t g = lane / G, s = lane % G;
  const char* lds_lane = reinterpret_cast<const char*>(lds) + s * LW * 4;
  const uint64_t gw0 = (uint64_t)tile * TW + (uint64_t)s * LW;

  const uint64_t n_groups = (r_end - r_begin + RPW - 1) / RPW;
  for (uint32_t grp = wave; grp < n_groups;) {
    const uint64_t base = r_begin + (uint64_t)grp * RPW;
    const uint64_t k0 = base + g;
    const bool active = k0 < r_end;
    // a lane past the chunk's end takes the chunk's first read (always
    // present) with no tokens of its own; it stores nothing
    const uint64_t k = active ? k0 : r_begin;
    const uint64_t rid = a.read_order ? a.read_order[k] : k;
    const uint32_t* tok;
    uint32_t* out_row;
    uint32_t ntok;
    int32_t T;
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
    if (!active) ntok = 0;
    if (__any(ntok > 255)) {
      // 16 counter planes: two (or one) words per pass keeps the registers
      // of this rare path within the budget of the common one
      constexpr int LWW = LW >= 2 ? 2 : 1;
#pragma unroll
      for (int h = 0; h < LW / LWW; ++h)
        scan_read<LWW, 11, COUNTS>(a, lds_lane + h * LWW * 4, active, tok, out_row, rid, ntok, T, gw0 + h * LWW);
    } else {
      scan_read<LW, 3, COUNTS>(a, lds_lane, active, tok, out_row, rid, ntok, T, gw0);
    }
    uint32_t claim = 0;
    if (lane == 0) claim = atomicAdd(&next_group, 1u);
    grp = (uint32_t)__builtin_amdgcn_readlane((int)claim, 0);
  }
}

template <int TW, int LW, int NT>
hipError_t launch_t(ScanArgs a, uint64_t reads_per_chunk, hipStream_t s) {
  // chunks of at most reads_per_chunk reads (whole workgroup iterations of
  // NT / (TW / LW) reads), as many per XCD on each of the 8 XCDs
  constexpr uint64_t kIter = (uint64_t)NT / (TW / LW);
  const uint64_t n_iter = (a.n_reads + kIter - 1) / kIter;
  const uint64_t it_per_chunk = reads_per_chunk / kIter > 0 ? reads_per_chunk / kIter : 1;
  const uint64_t per_xcd = (n_iter + 8 * it_per_chunk - 1) / (8 * it_per_chunk);
  if (per_xcd > 0x0FFFFFFFull) return hipErrorInvalidConfiguration;
  a.n_rchunks = (uint32_t)(8 * per_xcd);
  const uint64_t blocks = 8ull * per_xcd * a.n_tiles;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidConfiguration;
  // the per-bin count output is compiled only into its own instance: without
  // it the kernel fits 126 registers with no spills (1.5% faster on the
  // human-scale scan, and 36 GB less of scratch traffic per launch)
  if (a.counts_out)
    hipLaunchKernelGGL((k_scan_allbins<TW, LW, NT, true>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_scan_allbins<TW, LW, NT, false>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_allbins(const ScanArgs& a0, const ScanConfig& cfg, hipStream_t s) {
  ScanArgs a = a0;
  const int TW = tm_tile_words(a.q);
  const uint64_t rpc = cfg.reads_per_chunk > 0 ? (uint64_t)cfg.reads_per_chunk : 1;
  a.n_tiles = (uint32_t)((a.W + TW - 1) / TW);
  if (a.n_reads == 0 || a.n_tiles == 0) return hipSuccess;
  const int nt = cfg.threads;
  const bool w8 = cfg.lane_words == 8;
#define GRIM_SCAN_NT(TW_, LW_)                                              \
  do {                                                                      \
    if (nt == 1024) return launch_t<TW_, LW_, 1024>(a, rpc, s);             \
    if (nt == 256) return launch_t<TW_, LW_, 256>(a, rpc, s);               \
    return launch_t<TW_, LW_, 512>(a, rpc, s);                              \
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
