// Candidate-location filter (paper Section 3 steps 4-5): for each listed
// (read, bin) pair, count the read's tokens present in that bin's bit vector
// and compare with T_r.
//
// The count with multiplicity, sum_i bit[x][t_i], is rewritten as
// sum_j 2^j * popcount(vec_x AND plane_j), where plane_j is the 4^q-bit set of
// tokens whose number of occurrences in the read has bit j set. One
// wavefront handles one read: it counts the read's tokens straight into its
// multiplicity planes in LDS once, then each lane takes one candidate bin,
// streams that bin's vector (128 B at q=5, 512 B at q=6) from HBM with
// 16-byte loads and ANDs it with the planes (read from LDS with a
// wave-uniform address, i.e. a broadcast), counting with v_bcnt. The gather
// of one bin vector per pair is the compulsory traffic of this mode.
//
// Two lane layouts: one lane per pair (the lane streams the whole vector), or
// a group of G lanes per pair, each lane streaming 32 (q = 5) or 64 contiguous bytes
// of the vector (so one wavefront load touches 64/G vectors instead of 64
// scattered ones) with its slice of the planes kept in registers for all of
// the read's pairs, and the partial counts summed across the group with DPP
// moves.
//
// Two launch shapes: one wavefront per read (the hardware dispatcher
// balances), or a persistent grid whose wavefronts take the next reads from
// an atomic counter until none are left (reads of uneven length and candidate
// count in one launch, no per-wavefront dispatch cost, which bounds the
// short-list case: 4M wavefronts of ~1.4 us each leave most of the chip idle).

#include "grim_internal.h"

namespace grim {
namespace {

constexpr int kMaxPlanes = 16;  // multiplicities up to 65535

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of x over aligned groups of G lanes (G a power of two up to 32), left
// in every lane of the group. Within 16-lane rows the steps are DPP moves
// (swap neighbours, swap pairs, mirror the 8-lane halves, mirror the row);
// each step's partial sums are equal across the lanes they came from, so a
// mirror brings in the other half's sum.
template <int G>
__device__ __forceinline__ uint32_t group_sum(uint32_t x) {
  if constexpr (G >= 2) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  if constexpr (G >= 4) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  if constexpr (G >= 8) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
  if constexpr (G >= 16) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false); // row_mirror
  if constexpr (G >= 32) x += (uint32_t)__shfl_xor((int)x, 16);
  return x;
}

// Steps 1-3 for read r: the K multiplicity planes of its tokens in this
// wavefront's LDS, counted directly in bit-sliced form. Adding one occurrence
// of token t flips bit t of plane 0 with an atomic XOR; if the bit was set,
// the carry flips bit t of plane 1, and so on. The flips of one level commute,
// and level k + 1 is flipped once per 1 -> 0 transition of level k, i.e.
// floor(n_k / 2) times whatever the order of the lanes' atomics, so the planes
// end up holding every token's count in binary. K, the bit length of the
// largest count, is one more than the highest level any increment reached.
// Returns K, or -1 when the read has no candidates.
template <int VW>
__device__ __forceinline__ int build_planes(const CandArgs& a, uint64_t r, uint64_t n_cand, uint32_t* planes,
                                            uint32_t lane, int64_t* pc0, int64_t* pc1) {
  static_assert(VW <= 2048, "planes of 4^q bits, q <= 8");
  constexpr uint32_t kWords = kMaxPlanes * VW;
  const int64_t c0 = a.cand_off[r], c1 = a.cand_off[r + 1];
  if (c0 < 0 || c1 < c0 || (uint64_t)c1 > n_cand) {
    if (lane == 0) atomicOr(a.status, ST_BAD_CAND_OFF);
    return -1;
  }
  if (c0 == c1) return -1;
  *pc0 = c0;
  *pc1 = c1;
  const int64_t o0 = a.offsets[r], o1 = a.offsets[r + 1];
  const uint32_t ntok = (uint32_t)(o1 - o0 - a.q + 1);
  const uint32_t* tok = a.tokens + token_base(o0, r);
  const uint32_t R4 = a.R4;

  uint4* p4 = reinterpret_cast<uint4*>(planes);  // kWords = 16 VW, a multiple of 4
  for (uint32_t i = lane; i < kWords / 4; i += 64) p4[i] = make_uint4(0, 0, 0, 0);
  wave_sync();
  uint32_t top = 0;  // highest level reached + 1
  for (uint32_t i = lane; i < ntok; i += 64) {
    const uint32_t t = tok[i];
    if (t >= R4) continue;
    const uint32_t bit = 1u << (t & 31u);
    uint32_t* w = planes + (t >> 5);
    uint32_t k = 0;
    // a count stays below 2^16 (at most 65535 tokens), so k stays below kMaxPlanes
    while ((atomicXor(w + k * VW, bit) & bit) && k + 1 < (uint32_t)kMaxPlanes) ++k;
    top = max(top, k + 1);
  }
  for (int off = 32; off >= 1; off >>= 1) top = max(top, (uint32_t)__shfl_xor((int)top, off));
  wave_sync();
  return (int)top;
}

template <int VW>
__device__ __forceinline__ void cand_read(const CandArgs& a, uint64_t r, uint64_t n_cand,
                                          uint32_t* planes, uint32_t lane) {
  int64_t c0 = 0, c1 = 0;
  const int Ki = build_planes<VW>(a, r, n_cand, planes, lane, &c0, &c1);
  if (Ki < 0) return;
  const uint32_t K = (uint32_t)Ki;
  const int32_t T = a.thr[r];
  // 4. one candidate per lane
  for (int64_t cb = c0; cb < c1; cb += 64) {
    const int64_t c = cb + lane;
    if (c >= c1) break;
    const int32_t x = a.cand_bin[c];
    uint32_t cnt = 0;
    if (x < 0 || (uint64_t)x >= a.nb) {
      atomicOr(a.status, ST_BAD_BIN);
    } else {
      const uint32_t* vec = a.bm + (uint64_t)x * VW;
      uint32_t acc[4] = {0, 0, 0, 0};
      if constexpr (VW >= 4) {
        const uint4* v4 = reinterpret_cast<const uint4*>(vec);
#pragma unroll 8
        for (int w4 = 0; w4 < VW / 4; ++w4) {
          const uint4 v = v4[w4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if ((uint32_t)j < K) {
              const uint4 p = reinterpret_cast<const uint4*>(planes + j * VW)[w4];
              acc[j] += __popc(v.x & p.x) + __popc(v.y & p.y) + __popc(v.z & p.z) + __popc(v.w & p.w);
            }
          }
        }
        for (uint32_t j = 4; j < K; ++j) {  // rare: a token repeated 16 times or more
          uint32_t extra = 0;
          for (int w4 = 0; w4 < VW / 4; ++w4) {
            const uint4 v = v4[w4];
            const uint4 p = reinterpret_cast<const uint4*>(planes + j * VW)[w4];
            extra += __popc(v.x & p.x) + __popc(v.y & p.y) + __popc(v.z & p.z) + __popc(v.w & p.w);
          }
          cnt += extra << j;
        }
      } else {
        for (int w = 0; w < VW; ++w) {
          const uint32_t v = vec[w];
          for (uint32_t j = 0; j < K; ++j) cnt += (uint32_t)__popc(v & planes[j * VW + w]) << j;
        }
      }
      cnt += acc[0] + (acc[1] << 1) + (acc[2] << 2) + (acc[3] << 3);
    }
    if (a.count_out) a.count_out[c] = (uint16_t)cnt;
    if (a.pass_out) a.pass_out[c] = (int32_t)cnt >= T ? 1 : 0;
  }
  // the LDS of this wavefront is reused by its next read
  wave_sync();
}

// Cooperative layout: G = VW / WPL lanes per pair; lane j takes the 16-byte
// chunks j, G + j, 2G + j, ... (WPL words) of the bin's vector and keeps the
// same words of the first four planes in registers for all of the read's
// pairs. Each load instruction then covers G * 16 contiguous bytes of every
// vector it touches, so the texture units see whole 64-byte sectors instead
// of a quarter of one per lane. WPL is 8 for 32-word vectors (q = 5: fewer
// registers, more wavefronts in flight for the short candidate lists of that
// mode) and 16 above.
template <int VW>
__device__ __forceinline__ void cand_read_coop(const CandArgs& a, uint64_t r, uint64_t n_cand,
                                               uint32_t* planes, uint32_t lane) {
  constexpr int WPL = VW <= 32 ? 8 : 16;  // words of the vector per lane
  constexpr int G = VW / WPL;              // lanes per pair
  constexpr int PPW = 64 / G;              // pairs per wavefront pass
  int64_t c0 = 0, c1 = 0;
  const int Ki = build_planes<VW>(a, r, n_cand, planes, lane, &c0, &c1);
  if (Ki < 0) return;
  const uint32_t K = (uint32_t)Ki;
  const int32_t T = a.thr[r];
  const uint32_t j = lane % G, g = lane / G;
  uint32_t pl[4][WPL];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if ((uint32_t)k < K) {
#pragma unroll
      for (int w4 = 0; w4 < WPL / 4; ++w4) {
        const uint4 p = reinterpret_cast<const uint4*>(planes + k * VW)[w4 * G + j];
        pl[k][4 * w4 + 0] = p.x; pl[k][4 * w4 + 1] = p.y; pl[k][4 * w4 + 2] = p.z; pl[k][4 * w4 + 3] = p.w;
      }
    } else {
#pragma unroll
      for (int w = 0; w < WPL; ++w) pl[k][w] = 0;
    }
  }
  // U pair-passes per iteration: their bin ids, then their vectors, are
  // loaded together so that U gathers per lane are in flight at once
  constexpr int U = 2;
  for (int64_t cb = c0; cb < c1; cb += (int64_t)U * PPW) {
    int64_t c[U];
    int32_t x[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = cb + u * PPW + g;
      x[u] = c[u] < c1 ? a.cand_bin[c[u]] : 0;
    }
    uint32_t v[U][WPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = c[u] < c1 && x[u] >= 0 && (uint64_t)x[u] < a.nb;
      const uint4* v4 = reinterpret_cast<const uint4*>(a.bm + (uint64_t)(ok[u] ? x[u] : 0) * VW);
#pragma unroll
      for (int w4 = 0; w4 < WPL / 4; ++w4) {
        uint4 t = make_uint4(0, 0, 0, 0);
        if (ok[u]) t = v4[w4 * G + j];
        v[u][4 * w4 + 0] = t.x; v[u][4 * w4 + 1] = t.y; v[u][4 * w4 + 2] = t.z; v[u][4 * w4 + 3] = t.w;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint32_t part = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if ((uint32_t)k < K) {  // wave-uniform
          uint32_t acc = 0;
#pragma unroll
          for (int w = 0; w < WPL; ++w) acc += __popc(v[u][w] & pl[k][w]);
          part += acc << k;
        }
      }
      for (uint32_t k = 4; k < K; ++k) {  // rare: a token repeated 16 times or more
        uint32_t acc = 0;
        for (int w = 0; w < WPL; ++w) acc += __popc(v[u][w] & planes[k * VW + ((w / 4) * G + j) * 4 + w % 4]);
        part += acc << k;
      }
      part = group_sum<G>(part);  // the group's partial counts (groups are aligned runs of G lanes)
      if (j == 0 && c[u] < c1) {
        if (!ok[u]) {
          atomicOr(a.status, ST_BAD_BIN);
        } else {
          if (a.count_out) a.count_out[c[u]] = (uint16_t)part;
          if (a.pass_out) a.pass_out[c[u]] = (int32_t)part >= T ? 1 : 0;
        }
      }
    }
  }
  wave_sync();
}

// Four reads per wavefront (q = 5, 128-byte vectors): the lists of that
// mode are short (about 49 pairs per read on the 100 Mbp workload) and a
// read's steps are a chain of dependent loads (offsets, tokens, plane build,
// bin ids, vectors), so one read per wavefront leaves the chip waiting. Here
// each 16-lane quarter of a wavefront takes its own read: four reads' chains
// overlap, the plane builds of all four share the wavefront's two fences,
// and each quarter keeps U = 4 pair passes of 4 pairs in flight. Per read
// the steps are those of cand_read_coop: the planes are counted in LDS (16
// planes of 32 words per read), K comes from an LDS maximum, each lane holds
// words [8j, 8j + 8) of planes 0..3 in registers and ANDs them with the same
// words of each candidate bin's vector, and the 4 lanes of a pair sum their
// counts with DPP moves.
//
// NPL is the number of planes a read keeps in LDS: 16, or 8 for reads of at
// most 255 tokens (no count can reach 256). With 8, a read of more tokens is
// left to k_cand_long, and a wavefront's LDS halves (4 KB at q = 5), so LDS
// no longer limits how many wavefronts a CU holds.
constexpr int kQuadReads = 4;  // reads per wavefront in the quad layout

constexpr uint32_t kShortTokens = 255;  // most tokens of a read the 8-plane layout takes

template <int VW, int NPL>
__device__ __forceinline__ void cand_quad(const CandArgs& a, uint64_t r_first, uint64_t n_reads, uint64_t n_cand,
                                          uint32_t* planes_wave, uint32_t lane) {
  static_assert(VW == 32, "the quad layout is the q = 5 one");
  static_assert(NPL == 16 || NPL == 8, "planes per read");
  constexpr int WPL = 8, G = VW / WPL, QL = 64 / kQuadReads, PPQ = QL / G, U = G;
  constexpr uint32_t kPlaneWords = NPL * VW;
  const uint32_t qd = lane / QL, ql = lane % QL;
  const uint64_t r = r_first + qd;
  uint32_t* planes = planes_wave + qd * kPlaneWords;
  uint32_t* kword = planes_wave + kQuadReads * kPlaneWords + qd;  // largest level reached, per read
  int64_t c0 = 0, c1 = 0;
  uint32_t ntok = 0;
  int32_t T = 0;
  const uint32_t* tok = a.tokens;
  if (r < n_reads) {
    c0 = a.cand_off[r];
    c1 = a.cand_off[r + 1];
    if (c0 < 0 || c1 < c0 || (uint64_t)c1 > n_cand) {
      if (ql == 0) atomicOr(a.status, ST_BAD_CAND_OFF);
      c0 = c1 = 0;
    }
    const int64_t o0 = a.offsets[r];
    if (c1 > c0) ntok = (uint32_t)(a.offsets[r + 1] - o0 - a.q + 1);  // a read without pairs counts nothing
    if (NPL < kMaxPlanes && ntok > kShortTokens) c0 = c1 = ntok = 0;   // k_cand_long takes it
    tok = a.tokens + token_base(o0, r);
    T = a.thr[r];
  }
  uint4* p4 = reinterpret_cast<uint4*>(planes);
  for (uint32_t i = ql; i < kPlaneWords / 4; i += QL) p4[i] = make_uint4(0, 0, 0, 0);
  if (ql == 0) *kword = 0;
  wave_sync();
  const uint32_t R4 = a.R4;
  uint32_t top = 0;  // highest level reached + 1
  // four tokens per lane and load: a token list starts 16-byte aligned and its
  // padding (code R4) reaches past the next multiple of 4 above the count
  for (uint32_t i4 = ql * 4; i4 < ntok; i4 += 4 * QL) {
    const uint4 t4 = ldg4(tok + i4);
    const uint32_t tt[4] = {t4.x, t4.y, t4.z, t4.w};
    // the four level-0 flips are issued together; a token whose bit was
    // already set (a repeat) then carries into the levels above, in order
    uint32_t old[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      old[e] = tt[e] < R4 ? atomicXor(planes + (tt[e] >> 5), 1u << (tt[e] & 31u)) : 0u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t t = tt[e];
      if (t >= R4) continue;  // invalid window or padding
      const uint32_t bit = 1u << (t & 31u);
      uint32_t k = 0;
      if (old[e] & bit) {
        uint32_t* w = planes + (t >> 5);
        k = 1;
        // a count stays below 2^NPL (at most 65535 tokens, or 255 with 8 planes), so k stays below NPL
        while ((atomicXor(w + k * VW, bit) & bit) && k + 1 < (uint32_t)NPL) ++k;
      }
      top = max(top, k + 1);
    }
  }
  if (top) atomicMax(kword, top);
  wave_sync();
  const uint32_t K = *kword;
  const uint32_t j = ql % G, g = ql / G;
  constexpr int NR = 2;  // planes held in registers (counts below 4); higher ones are read from LDS
  uint32_t pl[NR][WPL];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if ((uint32_t)k < K) {
#pragma unroll
      for (int w4 = 0; w4 < WPL / 4; ++w4) {
        const uint4 p = reinterpret_cast<const uint4*>(planes + k * VW)[w4 * G + j];
        pl[k][4 * w4 + 0] = p.x; pl[k][4 * w4 + 1] = p.y; pl[k][4 * w4 + 2] = p.z; pl[k][4 * w4 + 3] = p.w;
      }
    } else {
#pragma unroll
      for (int w = 0; w < WPL; ++w) pl[k][w] = 0;
    }
  }
  // An iteration covers U = G passes of PPQ pairs: pair pb + u * PPQ + g of the
  // read goes to group g in pass u. Lane (g, j) loads the bin id of pass j and
  // stores the result of pass j, so each of those takes one instruction for
  // the whole wavefront; the bin ids reach the group's lanes by quad
  // broadcasts. Vectors are loaded unconditionally (bin 0 stands in for pairs
  // past the list's end and for bad bins, whose results are not stored), and
  // pair indices are 32-bit offsets within the read's list.
  const uint32_t npairs = (uint32_t)(c1 - c0);
  const int32_t* cbin = a.cand_bin + c0;
  uint16_t* cnt_out = a.count_out ? a.count_out + c0 : nullptr;
  uint8_t* pas_out = a.pass_out ? a.pass_out + c0 : nullptr;
  const uint32_t nb = (uint32_t)a.nb;  // at most 2^31 bins
  for (uint32_t pb = 0; pb < npairs; pb += U * PPQ) {
    const uint32_t pm = pb + j * PPQ + g;  // this lane's pair of pass j
    const bool livem = pm < npairs;
    const uint32_t xm = livem ? (uint32_t)cbin[pm] : 0u;
    const bool okm = xm < nb;             // a negative bin id is caught here too
    const uint32_t xs = okm ? xm : 0u;
    uint32_t x[U];
    x[0] = (uint32_t)__builtin_amdgcn_mov_dpp((int)xs, 0x00, 0xF, 0xF, false);  // quad_perm 0,0,0,0
    x[1] = (uint32_t)__builtin_amdgcn_mov_dpp((int)xs, 0x55, 0xF, 0xF, false);  // quad_perm 1,1,1,1
    x[2] = (uint32_t)__builtin_amdgcn_mov_dpp((int)xs, 0xAA, 0xF, 0xF, false);  // quad_perm 2,2,2,2
    x[3] = (uint32_t)__builtin_amdgcn_mov_dpp((int)xs, 0xFF, 0xF, 0xF, false);  // quad_perm 3,3,3,3
    // passes past every quarter's last pair (the short lists' final
    // iteration) load and count nothing: need[u] is the same in all lanes
    bool need[U];
    need[0] = true;
#pragma unroll
    for (int u = 1; u < U; ++u) need[u] = __any(npairs - pb > (uint32_t)u * PPQ);
    uint32_t v[U][WPL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!need[u]) continue;
      const uint4* v4 = reinterpret_cast<const uint4*>(a.bm) + (uint64_t)x[u] * (VW / 4);
#pragma unroll
      for (int w4 = 0; w4 < WPL / 4; ++w4) {
        const uint4 t = v4[w4 * G + j];
        v[u][4 * w4 + 0] = t.x; v[u][4 * w4 + 1] = t.y; v[u][4 * w4 + 2] = t.z; v[u][4 * w4 + 3] = t.w;
      }
    }
    uint32_t mine = 0;  // the group's count for pass j
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!need[u]) continue;
      uint32_t part = 0;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        if ((uint32_t)k < K) {
          uint32_t acc = 0;
#pragma unroll
          for (int w = 0; w < WPL; ++w) acc += __popc(v[u][w] & pl[k][w]);
          part += acc << k;
        }
      }
      for (uint32_t k = NR; k < K; ++k) {  // a token repeated 4 times or more
        uint32_t acc = 0;
        for (int w = 0; w < WPL; ++w) acc += __popc(v[u][w] & planes[k * VW + ((w / 4) * G + j) * 4 + w % 4]);
        part += acc << k;
      }
      part = group_sum<G>(part);
      if ((uint32_t)u == j) mine = part;
    }
    if (livem) {
      if (!okm) {
        atomicOr(a.status, ST_BAD_BIN);
      } else {
        if (cnt_out) cnt_out[pm] = (uint16_t)mine;
        if (pas_out) pas_out[pm] = (int32_t)mine >= T ? 1 : 0;
      }
    }
  }
  // the LDS of this wavefront is reused by its next reads
  wave_sync();
}

// LAYOUT: 0 one lane per pair, 1 VW/WPL lanes per pair, 2 four reads per
// wavefront (q = 5). A wavefront's "step" is one read, or four in layout 2.
template <int VW, int NW, bool PERSISTENT, int LAYOUT, int NPL>
__global__ __launch_bounds__(NW * 64) void k_scan_cand(CandArgs a) {
  // one region per wavefront: the multiplicity planes (NPL x VW words per read)
  static_assert(NPL == kMaxPlanes || LAYOUT == 2, "fewer planes only in the quad layout");
  constexpr uint32_t kReads = LAYOUT == 2 ? kQuadReads : 1;
  constexpr uint32_t kPerWave = kReads * NPL * VW + (LAYOUT == 2 ? kQuadReads : 0);
  __shared__ __attribute__((aligned(16))) uint32_t lds[NW * kPerWave];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  uint32_t* planes = lds + wave * kPerWave;
  const uint64_t n_reads = a.dyn ? min(a.dyn->n_reads, a.n_reads) : a.n_reads;
  const uint64_t n_cand = a.dyn ? min(a.dyn->n_cand, a.n_cand) : a.n_cand;
  if (a.status[0] & ~(uint32_t)(ST_BAD_BIN | ST_BAD_CAND_OFF)) return;  // rejected reads
  auto step = [&](uint64_t r) {
    if constexpr (LAYOUT == 2) cand_quad<VW, NPL>(a, r, n_reads, n_cand, planes, lane);
    else if constexpr (LAYOUT == 1) cand_read_coop<VW>(a, r, n_cand, planes, lane);
    else cand_read<VW>(a, r, n_cand, planes, lane);
  };
  if constexpr (!PERSISTENT) {
    const uint64_t r = ((uint64_t)blockIdx.x * NW + wave) * kReads;
    if (r < n_reads) step(r);
  } else {
    // every wavefront leaves once the counter has passed n_reads; reads are
    // taken a.grab at a time (a multiple of kReads) so the counter sees few atomics
    const uint32_t grab = a.grab;
    while (true) {
      uint32_t r0 = 0;
      if (lane == 0) r0 = atomicAdd(a.work, grab);
      r0 = __shfl(r0, 0);
      if ((uint64_t)r0 >= n_reads) break;
      const uint64_t r1 = min((uint64_t)r0 + grab, n_reads);
      for (uint64_t r = r0; r < r1; r += kReads) step(r);
    }
  }
}

// The reads of more than 255 tokens that the 8-plane quad layout leaves: each
// wavefront looks at 64 reads at a time (a lane each) and runs every long one
// that has pairs in the cooperative layout with all 16 planes.
template <int VW>
__global__ __launch_bounds__(256) void k_cand_long(CandArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[4 * kMaxPlanes * VW];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  uint32_t* planes = lds + wave * kMaxPlanes * VW;
  const uint64_t n_reads = a.dyn ? min(a.dyn->n_reads, a.n_reads) : a.n_reads;
  const uint64_t n_cand = a.dyn ? min(a.dyn->n_cand, a.n_cand) : a.n_cand;
  if (a.status[0] & ~(uint32_t)(ST_BAD_BIN | ST_BAD_CAND_OFF)) return;  // rejected reads
  const uint64_t stride = (uint64_t)gridDim.x * 4 * 64;
  for (uint64_t base = ((uint64_t)blockIdx.x * 4 + wave) * 64; base < n_reads; base += stride) {
    const uint64_t r = base + lane;
    bool is_long = false;
    if (r < n_reads) is_long = (uint64_t)(a.offsets[r + 1] - a.offsets[r]) > kShortTokens + a.q - 1;
    uint64_t m = __ballot(is_long);
    while (m) {
      const uint32_t l = (uint32_t)__builtin_ctzll(m);
      m &= m - 1;
      cand_read_coop<VW>(a, base + l, n_cand, planes, lane);
    }
  }
}

template <int VW, int NW, int LAYOUT, int NPL = kMaxPlanes>
hipError_t launch_nw_layout(const CandArgs& a, const CandConfig& cfg, hipStream_t s) {
  constexpr uint64_t kReads = LAYOUT == 2 ? kQuadReads : 1;
  const bool persistent = cfg.persistent == 1 || (cfg.persistent == 2 && a.n_reads >= kPersistentMinReads);
  if (persistent) {
    if (!a.work) return hipErrorInvalidValue;
    const uint64_t blocks = 256ull * (uint64_t)max(1, cfg.groups_per_cu);
    // about 8192 pairs per counter increment (64 reads of the short 100 Mbp
    // lists, ~49 pairs each; 8 of the 1024-pair uneven lists: measured best
    // for each), but at least four increments per wavefront of the grid
    CandArgs b = a;
    const uint64_t per_read = std::max<uint64_t>(1, a.n_cand / std::max<uint64_t>(1, a.n_reads));
    const uint64_t spread = a.n_reads / (4 * blocks * NW);
    uint64_t grab = std::min<uint64_t>(64, std::max<uint64_t>(1, std::min(8192 / per_read, spread)));
    b.grab = (uint32_t)((grab + kReads - 1) / kReads * kReads);
    hipError_t e = launch_zero_words(a.work, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scan_cand<VW, NW, true, LAYOUT, NPL>), dim3((unsigned)blocks), dim3(NW * 64), 0, s, b);
  } else {
    const uint64_t per_block = NW * kReads;
    const uint64_t blocks = (a.n_reads + per_block - 1) / per_block;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_scan_cand<VW, NW, false, LAYOUT, NPL>), dim3((unsigned)blocks), dim3(NW * 64), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if constexpr (NPL < kMaxPlanes) {
    // reads of more than 255 tokens, left by the 8-plane layout
    if (e != hipSuccess) return e;
    const uint64_t groups = std::min<uint64_t>(1024, (a.n_reads + 255) / 256);
    hipLaunchKernelGGL((k_cand_long<VW>), dim3((unsigned)groups), dim3(256), 0, s, a);
    e = hipGetLastError();
  }
  return e;
}

template <int VW, int NW>
hipError_t launch_nw(const CandArgs& a, const CandConfig& cfg, hipStream_t s) {
  if constexpr (VW == 32) {
    if (cfg.coop == 2) {
      if (cfg.planes == 16) return launch_nw_layout<VW, NW, 2>(a, cfg, s);
      return launch_nw_layout<VW, NW, 2, 8>(a, cfg, s);
    }
  }
  // the cooperative layout needs a pair's vector within one wavefront's lanes
  if constexpr (VW >= 32 && VW <= 512) {
    if (cfg.coop) return launch_nw_layout<VW, NW, 1>(a, cfg, s);
  }
  return launch_nw_layout<VW, NW, 0>(a, cfg, s);
}

// LDS per wavefront: 16 * VW words; the wave count per group is capped so a
// group stays within 64 KB, except at q = 8, where one wavefront's planes take
// 128 KB of the 160 KB of a CU: one wavefront per group and per CU, each lane
// streaming whole 8 KB vectors (a boundary case the paper's token lengths of
// 4 to 6 do not reach).
template <int VW>
hipError_t launch_vw(const CandArgs& a, const CandConfig& cfg, hipStream_t s) {
  constexpr int kMaxNW = VW >= 2048 ? 1 : (VW >= 512 ? 2 : 8);
  // default: 4 wavefronts per group where the pairs are gathered
  // cooperatively (measured best at q = 6), else as many as fit
  const int nw = cfg.waves > 0 ? cfg.waves : (VW >= 32 && VW < 512 && cfg.coop ? 4 : kMaxNW);
  if (nw >= 8 && kMaxNW >= 8) return launch_nw<VW, (kMaxNW >= 8 ? 8 : 1)>(a, cfg, s);
  if (nw >= 4 && kMaxNW >= 4) return launch_nw<VW, (kMaxNW >= 4 ? 4 : 1)>(a, cfg, s);
  if (nw >= 2 && kMaxNW >= 2) return launch_nw<VW, (kMaxNW >= 2 ? 2 : 1)>(a, cfg, s);
  return launch_nw<VW, 1>(a, cfg, s);
}

__global__ void k_zero_words(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_zero_words(uint32_t* p, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_scan_candidates(const CandArgs& a, const CandConfig& cfg, hipStream_t s) {
  if (a.n_reads == 0) return hipSuccess;
  switch (a.vec_words) {
    case 1: return launch_vw<1>(a, cfg, s);
    case 2: return launch_vw<2>(a, cfg, s);
    case 8: return launch_vw<8>(a, cfg, s);
    case 32: return launch_vw<32>(a, cfg, s);
    case 128: return launch_vw<128>(a, cfg, s);
    case 512: return launch_vw<512>(a, cfg, s);
    case 2048: return launch_vw<2048>(a, cfg, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace grim
