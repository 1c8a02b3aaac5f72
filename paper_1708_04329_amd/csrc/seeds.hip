// Seeding: the seed-and-extend steps that come before the filter (paper
// Section 1: a mapper picks seeds of a read, looks them up in an index of the
// reference, and obtains the candidate locations that the filter checks).
//
// Seed table. Every reference position p whose k bases are A, C, G or T is
// listed under the code of its k-mer: start[c] .. start[c + 1] index the
// positions of code c in pos[]. Built with one counting pass (atomic adds on
// the 4^k counters), an exclusive scan, and one filling pass that hands out
// slots by counting down.
//
// Candidates. A read's seeds are its non-overlapping k-mers at offsets 0, k,
// 2k, ...; a seed at offset o found at p votes for bin max(p - o, 0) / B. The
// read's candidates are its bins ranked by votes (more first), then by bin
// (smaller first), the first `cap` kept, listed by increasing bin. On the GPU:
//   1. hits per read (a thread per read: table lookups of its seeds);
//   2. reads are cut into batches whose staging (min(hits, cap) slots per
//      read) is bounded, and sorted by hit count into four table sizes;
//   3. a workgroup per read counts its bins' votes in an LDS hash table,
//      picks the kept bins (vote threshold from a histogram, ties by a radix
//      select on the bin) and writes them sorted to its staging slots;
//   4. the few reads a table cannot describe exactly take a slower path in
//      device memory (sort, runs, exact selection);
//   5. a scan of the kept counts gives the CSR offsets, and the lists move
//      from staging to their place.

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "grim_internal.h"

struct grim_seeds {
  int device = 0;
  uint64_t G = 0;
  uint32_t k = 0;
  uint64_t nk = 0;
  uint64_t* start = nullptr;  // [nk + 1]
  uint32_t* pos = nullptr;    // [n_pos]
  uint64_t n_pos = 0;
  std::mutex mu;
  // scratch of grim_seed_candidates (grown on demand)
  uint64_t* hits = nullptr;       // [n_reads] hits per read
  uint64_t* hits_host = nullptr;  // pinned copy
  uint64_t hits_cap = 0, hits_host_cap = 0;
  uint64_t* words = nullptr;      // [8]: CSR total so far (two words, by batch parity), bad offsets, fallback count
  uint32_t* tmp = nullptr;        // staging: kept bins per read
  uint64_t tmp_cap = 0;
  uint64_t* toff = nullptr;       // [batch reads] first staging slot
  uint64_t toff_cap = 0;
  uint64_t* outoff = nullptr;     // [batch reads] CSR offset
  uint64_t outoff_cap = 0;
  uint64_t* bsum = nullptr;       // scan block sums
  uint64_t bsum_cap = 0;
  uint32_t* cnt = nullptr;        // [batch reads] bins kept
  uint64_t cnt_cap = 0;
  uint32_t* list = nullptr;       // [batch reads] reads grouped by table size
  uint64_t list_cap = 0;
  uint32_t* redo = nullptr;       // [batch reads] reads for the fallback
  uint64_t redo_cap = 0;
  uint32_t* slab = nullptr;       // fallback work space
  uint64_t slab_cap = 0;
  uint64_t* toff_host = nullptr;  // pinned
  uint32_t* list_host = nullptr;  // pinned
  uint64_t host_cap = 0;
  uint8_t* staging = nullptr;     // host-resident reads copied in
  uint64_t staging_cap = 0;
  uint64_t* total_host = nullptr; // pinned [4]
};

namespace grim {
namespace {

struct SeedGuard {
  int prev = -1;
  explicit SeedGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~SeedGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

__device__ __forceinline__ int base_code(uint8_t c) {
  switch (c | 0x20) {  // ASCII letters folded to lower case
    case 'a': return 0;
    case 'c': return 1;
    case 'g': return 2;
    case 't': return 3;
    default: return -1;
  }
}

constexpr uint32_t kSpan = 64;  // reference positions per thread in the table passes

// Visit every valid k-mer starting in [p0, p0 + kSpan): f(code, p).
template <typename F>
__device__ __forceinline__ void for_kmers(const uint8_t* ref, uint64_t G, uint32_t k, uint64_t p0, F f) {
  const uint64_t mask = (k >= 32) ? ~0ull : ((1ull << (2 * k)) - 1ull);
  const uint64_t end = min(G, p0 + kSpan + k - 1);
  uint64_t code = 0;
  uint32_t run = 0;  // valid bases ending at i
  for (uint64_t i = p0; i < end; ++i) {
    const int c = base_code(ref[i]);
    if (c < 0) {
      run = 0;
      continue;
    }
    code = ((code << 2) | (uint64_t)c) & mask;
    if (++run >= k) f(code, i + 1 - k);
  }
}

// The same walk with the thread's bytes loaded up front: 80 bytes in five 16-byte loads (64
// start positions plus up to 13 more bases for k <= 14), the bases then coded without
// branches. Needs a 16-byte aligned reference; a thread whose 80 bytes run past the end takes
// the byte-wise walk.
template <typename F>
__device__ __forceinline__ void for_kmers_vec(const uint8_t* ref, uint64_t G, uint32_t k, uint64_t p0, F f) {
  constexpr uint32_t kBytes = 80;
  if (p0 + kBytes > G) {
    for_kmers(ref, G, k, p0, f);
    return;
  }
  uint4 v[kBytes / 16];
  const uint4* src = reinterpret_cast<const uint4*>(ref + p0);
#pragma unroll
  for (uint32_t j = 0; j < kBytes / 16; ++j) v[j] = src[j];
  const uint32_t* w = reinterpret_cast<const uint32_t*>(v);
  const uint64_t mask = (1ull << (2 * k)) - 1ull;  // k <= 14
  const uint32_t end = kSpan + k - 1;
  uint64_t code = 0;
  uint32_t run = 0;
#pragma unroll
  for (uint32_t i = 0; i < kBytes; ++i) {
    if (i >= end) break;
    const uint32_t d = (((w[i >> 2] >> (8 * (i & 3))) & 0xFFu) | 0x20u) - 0x60u;  // 'a' -> 1 ... 't' -> 20
    const bool ok = d < 32u && ((0x0010008Au >> d) & 1u);                        // a, c, g, t
    run = ok ? run + 1 : 0;
    code = ((code << 2) | (uint64_t)(((d >> 1) ^ (d >> 2)) & 3u)) & mask;       // a0 c1 g2 t3
    if (run >= k) f(code, p0 + i + 1 - k);
  }
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_kmer_count(const uint8_t* ref, uint64_t G, uint32_t k, uint32_t* counts) {
  const uint64_t p0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kSpan;
  if (p0 + k > G) return;
  auto visit = [&](uint64_t code, uint64_t) { atomicAdd(&counts[code], 1u); };
  if (VEC)
    for_kmers_vec(ref, G, k, p0, visit);
  else
    for_kmers(ref, G, k, p0, visit);
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_kmer_fill(const uint8_t* ref, uint64_t G, uint32_t k,
                                                   const uint64_t* start, uint32_t* counts, uint32_t* pos) {
  const uint64_t p0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kSpan;
  if (p0 + k > G) return;
  auto visit = [&](uint64_t code, uint64_t p) {
    const uint32_t left = atomicSub(&counts[code], 1u);  // in [1, count]
    pos[start[code] + left - 1] = (uint32_t)p;
  };
  if (VEC)
    for_kmers_vec(ref, G, k, p0, visit);
  else
    for_kmers(ref, G, k, p0, visit);
}

// Code of the k bases at s, or -1 if one is not A, C, G, T.
// The k <= 14 bases are all loaded before any is coded (the seed lies within
// its read), so their latencies overlap.
__device__ __forceinline__ int64_t seed_code(const uint8_t* s, uint32_t k) {
  uint8_t b[14];
#pragma unroll
  for (uint32_t j = 0; j < 14; ++j) b[j] = j < k ? s[j] : (uint8_t)'A';
  uint64_t code = 0;
  bool ok = true;
#pragma unroll
  for (uint32_t j = 0; j < 14; ++j) {
    if (j >= k) break;
    const int c = base_code(b[j]);
    ok = ok && c >= 0;
    code = (code << 2) | (uint64_t)(c & 3);
  }
  return ok ? (int64_t)code : -1;
}

// A read whose offsets are out of order or outside [0, n_bases] gets no hits
// and sets *bad; the call then fails before any later pass reads its bases.
__global__ __launch_bounds__(256) void k_seed_hits(const uint64_t* start, uint32_t k, const uint8_t* bases,
                                                   uint64_t n_bases, const int64_t* offsets, uint64_t n,
                                                   uint64_t* hits, uint32_t* bad) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t o0 = offsets[r], o1 = offsets[r + 1];
  if (o0 < 0 || o1 < o0 || (uint64_t)o1 > n_bases) {
    hits[r] = 0;
    atomicOr(bad, 1u);
    return;
  }
  const uint8_t* rd = bases + o0;
  const int64_t L = o1 - o0;
  uint64_t h = 0;
  for (int64_t o = 0; o + (int64_t)k <= L; o += k) {
    const int64_t c = seed_code(rd + o, k);
    if (c >= 0) h += start[c + 1] - start[c];
  }
  hits[r] = h;
}

// ---------------------------------------------------------------------------
// Exclusive prefix sums (uint32 in, uint64 out) in three passes: block sums,
// one workgroup scanning them (plus an optional base held in device memory),
// then each block's own elements.
// ---------------------------------------------------------------------------
constexpr uint32_t kScanT = 256, kScanV = 16, kScanBlock = kScanT * kScanV;

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, d);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), d);
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive scan over the workgroup (T threads); *total receives the sum.
template <int T, typename V>
__device__ __forceinline__ V block_excl_scan(V v, V* ws, V* total) {
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  V x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    V y;
    if constexpr (sizeof(V) == 8) y = shfl_up64(x, d);
    else y = (V)__shfl_up((int)x, d);
    if ((int)lane >= d) x += y;
  }
  if (lane == 63) ws[w] = x;
  __syncthreads();
  if (t == 0) {
    V run = 0;
    for (int i = 0; i < T / 64; ++i) {
      const V s = ws[i];
      ws[i] = run;
      run += s;
    }
    ws[T / 64] = run;
  }
  __syncthreads();
  const V r = ws[w] + x - v;
  *total = ws[T / 64];
  __syncthreads();  // ws is reused by the next call
  return r;
}

__global__ __launch_bounds__(kScanT) void k_scan_sums(const uint32_t* in, uint64_t n, uint64_t* bsum) {
  __shared__ uint64_t ws[kScanT / 64 + 1];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanBlock;
  uint64_t s = 0;
  for (uint64_t i = b0 + threadIdx.x; i < n && i < b0 + kScanBlock; i += kScanT) s += in[i];
  uint64_t total;
  (void)block_excl_scan<kScanT, uint64_t>(s, ws, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One workgroup: bsum[] becomes exclusive offsets (plus *base); *total_out = *base + sum.
__global__ __launch_bounds__(1024) void k_scan_top(uint64_t* bsum, uint64_t nblk, const uint64_t* base,
                                                   uint64_t* total_out) {
  __shared__ uint64_t ws[1024 / 64 + 1];
  uint64_t carry = base ? *base : 0;
  for (uint64_t c0 = 0; c0 < nblk; c0 += 1024) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t v = i < nblk ? bsum[i] : 0;
    uint64_t total;
    const uint64_t ex = block_excl_scan<1024, uint64_t>(v, ws, &total);
    if (i < nblk) bsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanT) void k_scan_apply(const uint32_t* in, uint64_t n, const uint64_t* boff,
                                                       uint64_t* out) {
  __shared__ uint64_t ws[kScanT / 64 + 1];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanV;
  uint32_t v[kScanV];
  uint64_t s = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanV; ++j) {
    v[j] = b0 + j < n ? in[b0 + j] : 0u;
    s += v[j];
  }
  uint64_t total;
  uint64_t run = boff[blockIdx.x] + block_excl_scan<kScanT, uint64_t>(s, ws, &total);
#pragma unroll
  for (uint32_t j = 0; j < kScanV; ++j) {
    if (b0 + j < n) out[b0 + j] = run;
    run += v[j];
  }
}

// out[i] = (*base or 0) + in[0] + ... + in[i - 1]; *total_out = (*base or 0) + sum of in.
// bsum needs scan_blocks(n) words.
uint64_t scan_blocks(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

hipError_t launch_scan(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* bsum, const uint64_t* base,
                       uint64_t* total_out, hipStream_t s) {
  const uint64_t nblk = scan_blocks(n);
  if (nblk) {
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nblk), dim3(kScanT), 0, s, in, n, bsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nblk, base, total_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !nblk) return e;
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nblk), dim3(kScanT), 0, s, in, n, bsum, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Candidate selection, one workgroup per read, in LDS.
//
// Each hit's bin goes into an open-addressing hash table of packed entries
// (bin << vb | votes, linear probing, atomic compare-and-swap to claim a
// slot, atomic add to vote). With the table complete, a vote histogram gives
// the read's distinct bins D. If D <= cap every bin is kept; otherwise the
// kept bins are those with more votes than a threshold vt plus, among the
// bins with exactly vt votes, the `need` smallest: the largest such bin is
// found by a radix select over the table (8 bits of the bin per pass). The
// kept bins are compacted to the front of the table, sorted with a bitonic
// network, and written to the read's staging slots.
//
// A read whose hits do not fit the largest table is taken in R ranges of
// bins, ascending: one pass over the ranges gathers the vote histogram, a
// second keeps each range's share (the tie budget running across ranges)
// and appends it. A range that fills its table restarts the read with twice
// the ranges.
//
// Reads the table cannot describe exactly go to the fallback below: a bin
// with 2^vb - 1 votes (the packed vote field would overflow), or a vote
// threshold of 256 or more.
// ---------------------------------------------------------------------------
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kVoteHist = 256;  // votes counted exactly below this

struct SelArgs {
  const uint64_t* start;
  const uint32_t* pos;
  uint32_t k;
  const uint8_t* bases;
  const int64_t* offsets;
  uint64_t r0;               // first read of the batch
  const uint64_t* hits;      // [n_reads] hits per read
  const uint64_t* tmp_off;   // [batch reads] first staging slot of each read
  uint32_t* tmp;             // staging: each read's kept bins, ascending
  uint32_t* cnt;             // [batch reads] bins kept
  uint32_t* redo;            // [batch reads] reads handed to the fallback
  uint32_t* n_redo;          // their number
  const uint32_t* list;      // batch-relative reads of this launch
  uint32_t n_list;
  uint32_t cap;
  uint32_t nbins;            // bins are below nbins
  uint32_t bin_bits;         // bits of nbins - 1
  uint32_t vb;               // vote bits of a table entry
  uint32_t dm, ds1, ds2;     // loc / B as (t + ((loc - t) >> ds1)) >> ds2, t = umulhi(dm, loc)
  uint32_t range_hits;       // hits per range for reads taken in ranges
  uint32_t force_ranges;     // take every read of the launch in ranges (tests)
};

__device__ __forceinline__ uint32_t hit_bin(uint32_t p, uint64_t o, const SelArgs& a) {
  const uint32_t loc = (uint64_t)p > o ? (uint32_t)(p - o) : 0u;
  const uint32_t t = __umulhi(a.dm, loc);
  return (t + ((loc - t) >> a.ds1)) >> a.ds2;
}

// Ascending bitonic sort of d[0, N), N a power of two, by a workgroup of T threads.
template <int T>
__device__ void bitonic_sort(uint32_t* d, uint32_t N) {
  for (uint32_t kk = 2; kk <= N; kk <<= 1) {
    for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
      for (uint32_t q = threadIdx.x; q < N / 2; q += T) {
        const uint32_t lo = ((q & ~(j - 1u)) << 1) | (q & (j - 1u));
        const uint32_t hi = lo | j;
        const uint32_t x = d[lo], y = d[hi];
        if ((x > y) == ((lo & kk) == 0)) {
          d[lo] = y;
          d[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Ascending bitonic sort of the 4T values x[] held by a workgroup of T
// threads, thread t holding elements 4t .. 4t + 3. Partners within a thread
// are swapped in registers, partners in another lane of the wavefront come
// by a lane shuffle, and only the stages whose partner is in another
// wavefront (distance 256 or more) go through LDS (buf, 4T words), with two
// barriers each: log2(T / 64) (log2(T / 64) + 1) / 2 + ... of the
// log2(4T) (log2(4T) + 1) / 2 stages, e.g. 3 of 55 for T = 256.
template <int T>
__device__ void bitonic_sort_regs(uint32_t (&x)[4], uint32_t* buf) {
  constexpr uint32_t N = 4 * T;
  const uint32_t t = threadIdx.x;
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      uint32_t y[4];
      if (j >= 256) {
        __syncthreads();  // every thread is done with buf
        *reinterpret_cast<uint4*>(buf + 4 * t) = make_uint4(x[0], x[1], x[2], x[3]);
        __syncthreads();
        const uint4 v = *reinterpret_cast<const uint4*>(buf + ((4 * t) ^ j));
        y[0] = v.x; y[1] = v.y; y[2] = v.z; y[3] = v.w;
      } else if (j >= 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) y[e] = (uint32_t)__shfl_xor((int)x[e], (int)(j >> 2));
      } else if (j == 2) {
        y[0] = x[2]; y[1] = x[3]; y[2] = x[0]; y[3] = x[1];
      } else {
        y[0] = x[1]; y[1] = x[0]; y[2] = x[3]; y[3] = x[2];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t i = 4 * t + (uint32_t)e;
        const bool take_min = ((i & k) == 0) == ((i & j) == 0);
        x[e] = take_min ? min(x[e], y[e]) : max(x[e], y[e]);
      }
    }
  }
}

// Inclusive scan over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, uint32_t lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, d);
    if ((int)lane >= d) x += y;
  }
  return x;
}

enum : uint32_t { kTiesNone = 0, kTiesAll = 1, kTiesUpTo = 2 };
enum : uint32_t { kModeAll = 0, kModeSelect = 1, kModeFallback = 2 };

template <int T, int SMAX>
__global__ __launch_bounds__(T) void k_seed_select(SelArgs a) {
  static_assert(SMAX % T == 0 && T % 64 == 0 && T <= 1024, "shape");
  __shared__ __attribute__((aligned(16))) uint32_t tab[SMAX];
  __shared__ uint32_t hist[kVoteHist + 1];  // [v]: bins with v votes; [256]: 256 or more
  __shared__ uint32_t dig[256];
  __shared__ uint32_t s_h0[T];
  __shared__ uint32_t s_pre[T + 1];
  __shared__ uint32_t ws[T / 64 + 1];
  // sh[0] slots claimed, [1] table at its limit, [2] vote field full,
  // [3] mode, [4] vt, [5] need, [6] ties at vt, [7] digit, [8] count below it
  __shared__ uint32_t sh[9];
  const uint32_t t = threadIdx.x, lane = t & 63u;
  const uint32_t vmask = (1u << a.vb) - 1u;
  for (uint32_t li = blockIdx.x; li < a.n_list; li += gridDim.x) {
    const uint32_t i = a.list[li];
    const uint64_t r = a.r0 + i;
    const uint64_t H = a.hits[r];
    if (t == 0) sh[2] = 0;  // read by no thread before the first clear()'s barrier
    const int64_t o0 = a.offsets[r];
    const uint8_t* rd = a.bases + o0;
    const uint32_t n_seeds = (uint32_t)((a.offsets[r + 1] - o0) / a.k);
    auto room = [](uint32_t s) { return min(s / 4u * 3u, s - (uint32_t)T - 1u); };
    uint32_t S = 2 * T;
    while (S < (uint32_t)SMAX && room(S) < H) S <<= 1;
    const uint32_t logS = 31u - __clz(S);
    const uint32_t limit = room(S);
    // A read with more hits than the largest table's room is first tried
    // whole, counting the slots it claims (its hits often share bins); only
    // if its distinct bins overflow the table is it taken in ranges.
    const bool counted = room(S) < H;
    auto ranges_for = [&]() {
      uint32_t r = (uint32_t)min<uint64_t>((H + a.range_hits - 1) / a.range_hits, 1u << 16);
      if (counted && r < 2) r = 2;
      return r == 0 ? 1u : r;
    };
    uint32_t R = a.force_ranges ? ranges_for() : 1u;

    auto clear = [&]() {
      __syncthreads();  // every thread is done with the table and the flags
      for (uint32_t s = t; s < S; s += T) tab[s] = kEmpty;
      if (t == 0) {
        sh[0] = 0;
        sh[1] = 0;
      }
      __syncthreads();
    };
    auto insert = [&](uint32_t bin) {
      uint32_t sl = (bin * 0x9E3779B1u) >> (32u - logS);
      while (true) {
        uint32_t e = tab[sl];
        if (e == kEmpty) {
          if (sh[1]) return;  // the table is at its limit: the read restarts
          e = atomicCAS(&tab[sl], kEmpty, (bin << a.vb) | 1u);
          if (e == kEmpty) {
            if (atomicAdd(&sh[0], 1u) + 1u >= limit) sh[1] = 1u;
            return;
          }
        }
        if ((e >> a.vb) == bin) {
          const uint32_t old = atomicAdd(&tab[sl], 1u);
          if ((old & vmask) + 1u >= vmask) sh[2] = 1u;
          return;
        }
        sl = (sl + 1u) & (S - 1u);
      }
    };
    // every hit whose bin lies in [lo, hi) into the table
    auto walk = [&](uint32_t lo, uint32_t hi) {
      for (uint32_t sc = 0; sc < n_seeds; sc += T) {
        const uint32_t ns = min((uint32_t)T, n_seeds - sc);
        uint32_t h0 = 0, c = 0;
        if (t < ns) {
          const int64_t code = seed_code(rd + (uint64_t)(sc + t) * a.k, a.k);
          if (code >= 0) {
            const uint64_t b = a.start[code];
            h0 = (uint32_t)b;
            c = (uint32_t)(a.start[code + 1] - b);
          }
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<T, uint32_t>(c, ws, &total);
        s_h0[t] = h0;
        s_pre[t] = ex;  // threads past the chunk's seeds hold the total
        if (t == 0) s_pre[T] = total;
        __syncthreads();
        // HB hits per thread at a time: their positions are loaded together,
        // so the loads' latencies overlap instead of following each insert
        constexpr uint32_t HB = 8;
        uint32_t s = 0;
        for (uint32_t f0 = t; f0 < total; f0 += HB * T) {
          uint32_t p[HB], o[HB];
#pragma unroll
          for (uint32_t h = 0; h < HB; ++h) {
            const uint32_t f = f0 + h * T;
            p[h] = 0;
            o[h] = 0;
            if (f < total) {
              while (s_pre[s + 1] <= f) ++s;
              p[h] = a.pos[s_h0[s] + (f - s_pre[s])];
              o[h] = (sc + s) * a.k;
            }
          }
#pragma unroll
          for (uint32_t h = 0; h < HB; ++h) {
            if (f0 + h * T >= total) break;
            const uint32_t bin = hit_bin(p[h], o[h], a);
            if (bin >= lo && bin < hi) insert(bin);
          }
        }
        __syncthreads();  // the seed arrays are rewritten by the next chunk
      }
      __syncthreads();
    };
    // Every hit into the table. Each lane works through its HB hits at its
    // own pace: one compare-and-swap per probe step, and a lane whose hit is
    // placed moves on to its next one, so the wavefront does not wait for its
    // slowest lane's probe chain at every hit. When the read's hits exceed the
    // table's room (counted), the slots claimed are counted, one atomic per
    // wavefront and step, and once the count reaches the limit no lane starts
    // another hit (at most T more slots are claimed, which leaves the table a
    // free slot, so every probe ends); sh[1] then tells the caller.
    auto walk_all = [&](bool counted) {
      for (uint32_t sc = 0; sc < n_seeds; sc += T) {
        const uint32_t ns = min((uint32_t)T, n_seeds - sc);
        uint32_t h0 = 0, c = 0;
        if (t < ns) {
          const int64_t code = seed_code(rd + (uint64_t)(sc + t) * a.k, a.k);
          if (code >= 0) {
            const uint64_t b = a.start[code];
            h0 = (uint32_t)b;
            c = (uint32_t)(a.start[code + 1] - b);
          }
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<T, uint32_t>(c, ws, &total);
        s_h0[t] = h0;
        s_pre[t] = ex;  // threads past the chunk's seeds hold the total
        if (t == 0) s_pre[T] = total;
        __syncthreads();
        constexpr uint32_t HB = 8;
        uint32_t s = 0;
        for (uint32_t f0 = t; f0 < total; f0 += HB * T) {
          uint32_t bins[HB];
          uint32_t nh = 0;  // this lane's hits in the batch: bins[0 .. nh)
#pragma unroll
          for (uint32_t h = 0; h < HB; ++h) {
            const uint32_t f = f0 + h * T;
            bins[h] = 0;
            if (f < total) {
              while (s_pre[s + 1] <= f) ++s;
              bins[h] = hit_bin(a.pos[s_h0[s] + (f - s_pre[s])], (uint64_t)(sc + s) * a.k, a);
              nh = h + 1;
            }
          }
          if (counted && sh[1]) nh = 0;
          uint32_t bin = bins[0];
          uint32_t sl = (bin * 0x9E3779B1u) >> (32u - logS);
          while (nh) {
            const uint32_t old = atomicCAS(&tab[sl], kEmpty, (bin << a.vb) | 1u);
            const bool claimed = old == kEmpty;
            bool placed = claimed;
            if (!placed && (old >> a.vb) == bin) {
              const uint32_t o2 = atomicAdd(&tab[sl], 1u);
              if ((o2 & vmask) + 1u >= vmask) sh[2] = 1u;
              placed = true;
            }
            if (counted) {
              const uint64_t m = __ballot(claimed);
              if (m && lane == (uint32_t)__builtin_ctzll(m)) {
                const uint32_t nc = (uint32_t)__popcll(m);
                if (atomicAdd(&sh[0], nc) + nc >= limit) sh[1] = 1u;
              }
            }
            if (placed) {
              --nh;
#pragma unroll
              for (uint32_t h = 0; h + 1 < HB; ++h) bins[h] = bins[h + 1];
              bin = bins[0];
              sl = (bin * 0x9E3779B1u) >> (32u - logS);
              if (counted && sh[1]) nh = 0;
            } else {
              sl = (sl + 1u) & (S - 1u);
            }
          }
        }
        __syncthreads();  // the seed arrays are rewritten by the next chunk
      }
      __syncthreads();
    };
    // hist[] += the votes of the table's entries
    auto histo = [&]() {
      uint32_t n1 = 0, n2 = 0;
      for (uint32_t sl = t; sl < S; sl += T) {  // S is a multiple of T
        const uint32_t e = tab[sl];
        const uint32_t v = e == kEmpty ? 0u : (e & vmask);
        n1 += (uint32_t)__popcll(__ballot(v == 1u));
        n2 += (uint32_t)__popcll(__ballot(v == 2u));
        if (v > 2u) atomicAdd(&hist[min(v, kVoteHist)], 1u);
      }
      if (lane == 0) {
        atomicAdd(&hist[1], n1);
        atomicAdd(&hist[2], n2);
      }
      __syncthreads();
    };
    auto zero_hist = [&]() {
      for (uint32_t v = t; v <= kVoteHist; v += T) hist[v] = 0;
      __syncthreads();
    };
    // mode, vt, need and ties from hist (wavefront 0; lane l holds votes 4l .. 4l + 3)
    auto decide = [&]() {
      if (t < 64) {
        uint32_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h[j] = hist[4 * lane + j];
        const uint32_t top = hist[kVoteHist];
        const uint32_t mine = h[0] + h[1] + h[2] + h[3];
        // bins with more votes than this lane's range, and the total
        const uint32_t incl = wave_incl_scan(mine, lane);
        const uint32_t all = (uint32_t)__shfl((int)incl, 63) + top;
        const uint32_t above = all - incl;  // votes > 4 lane + 3 (hist[0] is 0)
        uint32_t vt = 0, run_vt = 0;
        uint32_t run = above;
        for (int j = 3; j >= 0; --j) {  // ge(4 lane + j) = run + h[j]
          const uint32_t v = 4 * lane + (uint32_t)j;
          if (!vt && v >= 1 && run + h[j] >= a.cap) {
            vt = v;
            run_vt = run;  // bins with more than vt votes
          }
          run += h[j];
        }
        // the largest vt: the highest lane that found one
        const uint64_t m = __ballot(vt != 0);
        if (lane == 0) {
          if (all <= a.cap) {
            sh[3] = kModeAll;
          } else if (top >= a.cap || m == 0) {
            sh[3] = kModeFallback;
          } else {
            sh[3] = kModeSelect;
          }
        }
        if (m != 0 && lane == 63u - (uint32_t)__clzll(m)) {
          sh[4] = vt;
          sh[5] = a.cap - run_vt;
          sh[6] = hist[vt];
        }
      }
      __syncthreads();
    };
    // the want-th smallest bin among the entries with vt votes (radix select, 8 bits a pass)
    auto select_bin = [&](uint32_t vt, uint32_t want) -> uint32_t {
      uint32_t prefix = 0;
      for (int hi = (int)a.bin_bits; hi > 0;) {
        const int w = hi < 8 ? hi : 8, s = hi - w;
        for (uint32_t d = t; d < 256; d += T) dig[d] = 0;
        __syncthreads();
        for (uint32_t sl = t; sl < S; sl += T) {
          const uint32_t e = tab[sl];
          if (e == kEmpty || (e & vmask) != vt) continue;
          const uint32_t bin = e >> a.vb;
          if (hi < 32 && (bin >> hi) != (prefix >> hi)) continue;
          atomicAdd(&dig[(bin >> s) & ((1u << w) - 1u)], 1u);
        }
        __syncthreads();
        if (t < 64) {
          uint32_t c[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) c[j] = dig[4 * lane + j];
          const uint32_t sum = c[0] + c[1] + c[2] + c[3];
          const uint32_t incl = wave_incl_scan(sum, lane);
          uint32_t cum = incl - sum;
          if (cum < want && want <= incl) {
            uint32_t d = 4 * lane;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              if (cum + c[j] >= want) break;
              cum += c[j];
              ++d;
            }
            sh[7] = d;
            sh[8] = cum;
          }
        }
        __syncthreads();
        prefix |= sh[7] << s;
        want -= sh[8];
        hi = s;
      }
      return prefix;
    };
    // the kept entries of the table (all, or more than vt votes plus the ties the rule admits),
    // ascending, to tmp[out_at ..]; returns their number
    auto emit = [&](bool all, uint32_t vt, uint32_t ties, uint32_t bt, uint64_t out_at) -> uint32_t {
      // every slot of the thread read into registers and tested, one scan for
      // the kept entries' places, which are then compacted to the table's front
      constexpr uint32_t SPT = SMAX / T;  // most slots per thread
      const uint32_t spt = S / T;
      uint32_t ev[SPT];
      uint32_t nk = 0;
#pragma unroll
      for (uint32_t u = 0; u < SPT; ++u) {
        uint32_t e = kEmpty;
        if (u < spt) {
          e = tab[u * T + t];
          bool keep = false;
          if (e != kEmpty) {
            const uint32_t v = e & vmask;
            keep = all || v > vt || (v == vt && (ties == kTiesAll || (ties == kTiesUpTo && (e >> a.vb) <= bt)));
          }
          e = keep ? e >> a.vb : kEmpty;
        }
        ev[u] = e;
        nk += e != kEmpty ? 1u : 0u;
      }
      uint32_t K;
      uint32_t p = block_excl_scan<T, uint32_t>(nk, ws, &K);  // every slot has been read
#pragma unroll
      for (uint32_t u = 0; u < SPT; ++u)
        if (ev[u] != kEmpty) tab[p++] = ev[u];
      __syncthreads();
      if (K <= 4 * T) {
        // up to four entries per thread: sorted in registers, stored from there
        uint32_t x[4];
        const uint4 v = *reinterpret_cast<const uint4*>(tab + 4 * t);
        x[0] = 4 * t + 0 < K ? v.x : kEmpty;
        x[1] = 4 * t + 1 < K ? v.y : kEmpty;
        x[2] = 4 * t + 2 < K ? v.z : kEmpty;
        x[3] = 4 * t + 3 < K ? v.w : kEmpty;
        bitonic_sort_regs<T>(x, tab);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (4 * t + (uint32_t)e < K) a.tmp[out_at + 4 * t + e] = x[e];
        return K;
      }
      const uint32_t N = 1u << (32 - __clz(K - 1u));  // K > 4T >= 256
      for (uint32_t q = K + t; q < N; q += T) tab[q] = kEmpty;
      __syncthreads();
      bitonic_sort<T>(tab, N);
      for (uint32_t q = t; q < K; q += T) a.tmp[out_at + q] = tab[q];
      return K;
    };

    const uint64_t out0 = a.tmp_off[i];
    bool fallback = false;
    uint32_t kept = 0;
    if (R == 1) {
      clear();
      walk_all(counted);
      if (sh[1]) {
        R = ranges_for();  // its distinct bins overflowed the table
      } else if (sh[2]) {
        fallback = true;
      } else {
        zero_hist();
        histo();
        decide();
        const uint32_t mode = sh[3];
        if (mode == kModeFallback) {
          fallback = true;
        } else if (mode == kModeAll) {
          kept = emit(true, 0, kTiesNone, 0, out0);
        } else {
          const uint32_t vt = sh[4], need = sh[5], ties = sh[6];
          if (need < ties) kept = emit(false, vt, kTiesUpTo, select_bin(vt, need), out0);
          else kept = emit(false, vt, kTiesAll, 0, out0);
        }
      }
    }
    if (R > 1) {
      const uint64_t nbins = a.nbins;
      while (true) {
        const uint64_t W = (nbins + R - 1) / R;
        auto lo_of = [&](uint32_t j) { return (uint32_t)min<uint64_t>((uint64_t)j * W, 0xFFFFFFFFull); };
        auto hi_of = [&](uint32_t j) { return (uint32_t)min<uint64_t>((uint64_t)(j + 1) * W, 0xFFFFFFFFull); };
        // pass 1: the vote histogram over every range
        zero_hist();
        bool restart = false;
        for (uint32_t j = 0; j < R && !restart && !fallback; ++j) {
          clear();
          walk(lo_of(j), hi_of(j));
          if (sh[1]) restart = true;
          else if (sh[2]) fallback = true;
          else histo();
        }
        if (fallback) break;
        if (restart) {
          if (R >= (1u << 16)) {
            fallback = true;
            break;
          }
          R *= 2;
          continue;
        }
        decide();
        const uint32_t mode = sh[3];
        if (mode == kModeFallback) {
          fallback = true;
          break;
        }
        const uint32_t vt = sh[4];
        uint32_t need_left = mode == kModeSelect ? sh[5] : 0;
        const bool cut = mode == kModeSelect && sh[5] < sh[6];
        // pass 2: each range's kept bins, appended in bin order
        kept = 0;
        for (uint32_t j = 0; j < R; ++j) {
          clear();
          walk(lo_of(j), hi_of(j));
          if (mode == kModeAll) {
            kept += emit(true, 0, kTiesNone, 0, out0 + kept);
            continue;
          }
          if (!cut) {
            kept += emit(false, vt, kTiesAll, 0, out0 + kept);
            continue;
          }
          zero_hist();
          histo();
          const uint32_t ties_here = hist[vt];
          __syncthreads();
          if (need_left == 0) {
            kept += emit(false, vt, kTiesNone, 0, out0 + kept);
          } else if (ties_here <= need_left) {
            kept += emit(false, vt, kTiesAll, 0, out0 + kept);
            need_left -= ties_here;
          } else {
            kept += emit(false, vt, kTiesUpTo, select_bin(vt, need_left), out0 + kept);
            need_left = 0;
          }
        }
        break;
      }
    }
    if (t == 0) {
      if (fallback) {
        a.cnt[i] = 0;
        a.redo[atomicAdd(a.n_redo, 1u)] = i;
      } else {
        a.cnt[i] = kept;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fallback, one wavefront per read: every hit's bin into the wavefront's slab
// of device memory, a bitonic sort there, runs of equal bins become (bin,
// votes), and the kept runs are chosen exactly (vote threshold by counting,
// ties by bin).
// ---------------------------------------------------------------------------

// Votes of run j of a read whose runs start at rs[0 .. nr) within [0, s1).
__device__ __forceinline__ uint32_t run_votes(const uint32_t* rs, uint32_t j, uint32_t nr, uint32_t s1) {
  return (j + 1 < nr ? rs[j + 1] : s1) - rs[j];
}

// Runs with at least v votes, over the wavefront.
__device__ __forceinline__ uint32_t count_at_least(const uint32_t* rs, uint32_t nr, uint32_t s1, uint32_t v,
                                                   uint32_t lane) {
  uint32_t c = 0;
  for (uint32_t j0 = 0; j0 < nr; j0 += 64) {
    const uint32_t j = j0 + lane;
    c += (uint32_t)__popcll(__ballot(j < nr && run_votes(rs, j, nr, s1) >= v));
  }
  return c;
}

__global__ __launch_bounds__(64) void k_seed_fallback(SelArgs a, uint32_t* slab, uint64_t slab_words) {
  const uint32_t lane = threadIdx.x;
  uint32_t* keys = slab + (uint64_t)blockIdx.x * slab_words;
  const uint32_t n_redo = *a.n_redo;
  for (uint32_t jr = blockIdx.x; jr < n_redo; jr += gridDim.x) {
    const uint32_t i = a.redo[jr];
    const uint64_t r = a.r0 + i;
    const uint32_t H = (uint32_t)a.hits[r];
    const uint32_t N = H <= 1 ? H : 1u << (32 - __clz(H - 1u));
    uint32_t* rs = keys + N;  // run starts
    uint32_t* rb = rs + H;    // run bins
    const int64_t o0 = a.offsets[r];
    const uint8_t* rd = a.bases + o0;
    const uint32_t n_seeds = (uint32_t)((a.offsets[r + 1] - o0) / a.k);
    // 1. every hit's bin, seed by seed (64 seeds' ranges looked up at once)
    uint32_t w = 0;
    for (uint32_t sb = 0; sb < n_seeds; sb += 64) {
      uint64_t h0 = 0, h1 = 0;
      if (sb + lane < n_seeds) {
        const int64_t c = seed_code(rd + (uint64_t)(sb + lane) * a.k, a.k);
        if (c >= 0) {
          h0 = a.start[c];
          h1 = a.start[c + 1];
        }
      }
      const uint32_t m = min(64u, n_seeds - sb);
      for (uint32_t j = 0; j < m; ++j) {
        const uint32_t H0 = (uint32_t)__shfl((int)(uint32_t)h0, (int)j);
        const uint32_t H1 = (uint32_t)__shfl((int)(uint32_t)h1, (int)j);
        const uint64_t o = (uint64_t)(sb + j) * a.k;
        for (uint32_t h = H0 + lane; h < H1; h += 64) keys[w + (h - H0)] = hit_bin(a.pos[h], o, a);
        w += H1 - H0;
      }
    }
    for (uint32_t q = H + lane; q < N; q += 64) keys[q] = kEmpty;
    __syncthreads();
    // 2. sort
    bitonic_sort<64>(keys, N);
    // 3. runs of equal bins
    uint32_t nr = 0;
    for (uint32_t c0 = 0; c0 < H; c0 += 64) {
      const uint32_t idx = c0 + lane;
      const bool valid = idx < H;
      const uint32_t key = valid ? keys[idx] : 0u;
      const bool st = valid && (idx == 0 || keys[idx - 1] != key);
      const uint64_t mk = __ballot(st);
      if (st) {
        const uint32_t j = nr + (uint32_t)__popcll(mk & ((1ull << lane) - 1ull));
        rs[j] = idx;
        rb[j] = key;
      }
      nr += (uint32_t)__popcll(mk);
    }
    __syncthreads();
    // 4. the kept runs, in bin order
    uint32_t* out = a.tmp + a.tmp_off[i];
    if (nr <= a.cap) {
      for (uint32_t j = lane; j < nr; j += 64) out[j] = rb[j];
      if (lane == 0) a.cnt[i] = nr;
      __syncthreads();
      continue;
    }
    // the largest v with at least cap runs of >= v votes (bisection; votes <= H)
    uint32_t lo = 1, hi = H;
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo + 1) / 2;
      if (count_at_least(rs, nr, H, mid, lane) >= a.cap) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t vt = lo;
    const uint32_t need = a.cap - count_at_least(rs, nr, H, vt + 1, lane);
    uint32_t taken = 0, ties = 0;
    for (uint32_t j0 = 0; j0 < nr; j0 += 64) {
      const uint32_t j = j0 + lane;
      const uint32_t v = j < nr ? run_votes(rs, j, nr, H) : 0u;
      const bool tie = j < nr && v == vt;
      const uint64_t tm = __ballot(tie);
      const uint32_t tie_rank = ties + (uint32_t)__popcll(tm & ((1ull << lane) - 1ull));
      const bool keep = j < nr && (v > vt || (tie && tie_rank < need));
      const uint64_t km = __ballot(keep);
      if (keep) out[taken + (uint32_t)__popcll(km & ((1ull << lane) - 1ull))] = rb[j];
      taken += (uint32_t)__popcll(km);
      ties += (uint32_t)__popcll(tm);
    }
    if (lane == 0) a.cnt[i] = a.cap;
    __syncthreads();
  }
}

__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Each read's kept bins from the staging slots to their place in the CSR
// output (one wavefront per read); outoff already holds the absolute offsets.
__global__ __launch_bounds__(256) void k_seed_place(const uint64_t* tmp_off, const uint32_t* tmp, const uint32_t* cnt,
                                                    const uint64_t* outoff, uint64_t nb, uint64_t r0,
                                                    int64_t* cand_off, int32_t* cand_bin) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t i = wave_uniform((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (i >= nb) return;
  const uint64_t o = outoff[i];
  if (lane == 0) cand_off[r0 + i] = (int64_t)o;
  const uint32_t K = cnt[i];
  const uint32_t* src = tmp + tmp_off[i];
  for (uint32_t j = lane; j < K; j += 64) cand_bin[o + j] = (int32_t)src[j];
}

__global__ __launch_bounds__(256) void k_revcomp(const uint8_t* in, uint64_t n_bases, const int64_t* offsets, uint64_t n,
                                                  uint8_t* out, uint32_t* bad) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t r = wave_uniform((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (r >= n) return;
  const int64_t o0 = offsets[r], o1 = offsets[r + 1];
  if (o0 < 0 || o1 < o0 || (uint64_t)o1 > n_bases) {  // leave the read alone, flag the call
    if (lane == 0) atomicOr(bad, 1u);
    return;
  }
  const int64_t L = o1 - o0;
  for (int64_t i = lane; i < L; i += 64) {
    const uint8_t c = in[o0 + L - 1 - i];
    uint8_t d = c;
    switch (c) {
      case 'A': d = 'T'; break;
      case 'C': d = 'G'; break;
      case 'G': d = 'C'; break;
      case 'T': d = 'A'; break;
      case 'a': d = 't'; break;
      case 'c': d = 'g'; break;
      case 'g': d = 'c'; break;
      case 't': d = 'a'; break;
      default: break;
    }
    out[o0 + i] = d;
  }
}

__global__ void k_fill_word(uint32_t* p, uint32_t v) { *p = v; }

hipError_t launch_fill_word(uint32_t* p, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_word, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

template <typename T>
int grow_dev(T** p, uint64_t* cap, uint64_t need) {
  if (*cap >= need && *p) return GRIM_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const uint64_t n = need + need / 8 + 64;
  void* q = nullptr;
  GRIM_HIP_TRY(hipMalloc(&q, n * sizeof(T)));
  *p = static_cast<T*>(q);
  *cap = n;
  return GRIM_OK;
}

void free_seeds(grim_seeds* sd) {
  if (!sd) return;
  SeedGuard g(sd->device);
  for (void* p : {(void*)sd->start, (void*)sd->pos, (void*)sd->hits, (void*)sd->words, (void*)sd->tmp,
                  (void*)sd->toff, (void*)sd->outoff, (void*)sd->bsum, (void*)sd->cnt, (void*)sd->list,
                  (void*)sd->redo, (void*)sd->slab, (void*)sd->staging})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)sd->hits_host, (void*)sd->total_host, (void*)sd->toff_host, (void*)sd->list_host})
    if (p) (void)hipHostFree(p);
  delete sd;
}

// Staging slots per batch of the candidate passes, 4 bytes each
// (GRIM_SEED_BATCH_KEYS overrides, e.g. to exercise many batches in tests).
uint64_t batch_keys() {
  if (const char* e = std::getenv("GRIM_SEED_BATCH_KEYS")) {
    const long long v = std::atoll(e);
    if (v > 0) return (uint64_t)v;
  }
  return 1ull << 28;
}

// Test switches: route reads to the larger tables, to bin ranges, or to the fallback.
int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e && *e ? std::atoi(e) : dflt;
}
bool env_flag(const char* name) { return env_int(name, 0) != 0; }

// Table size class of a read with h hits (h <= the class's 3/4-full table).
// Table sizes (threads, entries): a class's table holds its reads' hits at
// most 3/4 full; smaller tables leave room for more workgroups per CU.
constexpr uint32_t kSeedClasses = 6;
uint32_t seed_class(uint64_t h) {
  return h <= 768 ? 0u : h <= 1536 ? 1u : h <= 3072 ? 2u : h <= 6144 ? 3u : h <= 12288 ? 4u : 5u;
}

// n / d for every 32-bit n as (t + ((n - t) >> s1)) >> s2 with t = umulhi(m, n)
// (the round-up multiplier method of Granlund and Montgomery, 1994).
void make_div(uint32_t d, uint32_t* m, uint32_t* s1, uint32_t* s2) {
  if (d == 1) {
    *m = 0;
    *s1 = 0;
    *s2 = 0;
    return;
  }
  const uint32_t l = 32u - (uint32_t)__builtin_clz(d - 1);  // ceil(log2 d)
  *m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  *s1 = 1;
  *s2 = l - 1;
}

}  // namespace
}  // namespace grim

using namespace grim;

extern "C" {

int grim_seeds_build(const uint8_t* ref, uint64_t ref_len, uint32_t ref_on_device, uint32_t k, void* hip_stream,
                     grim_seeds** out) {
  clear_error();
  if (!out) return set_error(GRIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ref) return set_error(GRIM_EINVAL, "ref is NULL");
  if (k < 1 || k > 14) return set_error(GRIM_EINVAL, "k must be in [1, 14]");
  if (ref_len < k) return set_error(GRIM_EINVAL, "reference shorter than k");
  if (ref_len > 0xFFFFFFFFull) return set_error(GRIM_EINVAL, "reference longer than 2^32 - 1 bases");
  if (ref_on_device > 1) return set_error(GRIM_EINVAL, "ref_on_device must be 0 or 1");
  int dev = 0;
  GRIM_HIP_TRY(hipGetDevice(&dev));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::unique_ptr<grim_seeds, void (*)(grim_seeds*)> sd(new grim_seeds, free_seeds);
  sd->device = dev;
  sd->G = ref_len;
  sd->k = k;
  sd->nk = 1ull << (2 * k);
  const uint8_t* dref = ref;
  uint8_t* staging = nullptr;
  uint32_t* counts = nullptr;
  void* tmp = nullptr;
  auto cleanup = [&]() {
    if (staging) (void)hipFree(staging);
    if (counts) (void)hipFree(counts);
    if (tmp) (void)hipFree(tmp);
  };
  auto fail = [&](hipError_t e, const char* what) {
    cleanup();
    return set_error(e == hipErrorOutOfMemory ? GRIM_ENOMEM : GRIM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  if (!ref_on_device) {
    if ((e = hipMalloc(&staging, ref_len)) != hipSuccess) return fail(e, "reference staging");
    if ((e = hipMemcpyAsync(staging, ref, ref_len, hipMemcpyHostToDevice, s)) != hipSuccess)
      return fail(e, "reference copy");
    dref = staging;
  }
  if ((e = hipMalloc(&counts, (sd->nk + 1) * sizeof(uint32_t))) != hipSuccess) return fail(e, "k-mer counts");
  if ((e = hipMalloc(&sd->start, (sd->nk + 1) * sizeof(uint64_t))) != hipSuccess) return fail(e, "k-mer starts");
  if ((e = launch_zero_words(counts, (uint32_t)(sd->nk + 1), s)) != hipSuccess) return fail(e, "zero counts");
  const uint64_t threads = (ref_len + kSpan - 1) / kSpan;
  const uint64_t blocks = (threads + 255) / 256;
  const bool vec = ((uintptr_t)dref & 15u) == 0;
  hipLaunchKernelGGL(vec ? k_kmer_count<true> : k_kmer_count<false>, dim3((unsigned)blocks), dim3(256), 0, s, dref,
                     ref_len, k, counts);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "k-mer count");
  if ((e = hipMalloc(&tmp, (scan_blocks(sd->nk + 1) + 1) * sizeof(uint64_t))) != hipSuccess)
    return fail(e, "scan storage");
  if ((e = launch_scan(counts, sd->nk + 1, sd->start, static_cast<uint64_t*>(tmp), nullptr, nullptr, s)) !=
      hipSuccess)
    return fail(e, "k-mer scan");
  uint64_t n_pos = 0;
  if ((e = hipMemcpyAsync(&n_pos, sd->start + sd->nk, sizeof n_pos, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(e, "position count");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "position count");
  sd->n_pos = n_pos;
  if ((e = hipMalloc(&sd->pos, std::max<uint64_t>(n_pos, 1) * sizeof(uint32_t))) != hipSuccess)
    return fail(e, "positions");
  hipLaunchKernelGGL(vec ? k_kmer_fill<true> : k_kmer_fill<false>, dim3((unsigned)blocks), dim3(256), 0, s, dref,
                     ref_len, k, sd->start, counts, sd->pos);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "k-mer fill");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "k-mer fill");
  cleanup();
  *out = sd.release();
  return GRIM_OK;
}

int grim_seeds_info(const grim_seeds* sd, grim_seeds_info_t* out) {
  clear_error();
  if (!sd || !out) return set_error(GRIM_EINVAL, "NULL argument");
  out->ref_len = sd->G;
  out->k = sd->k;
  out->device = sd->device;
  out->n_positions = sd->n_pos;
  out->table_bytes = (sd->nk + 1) * sizeof(uint64_t) + sd->n_pos * sizeof(uint32_t);
  return GRIM_OK;
}

void grim_seeds_free(grim_seeds* sd) { free_seeds(sd); }

int grim_seed_candidates(const grim_seeds* csd, const grim_reads* rd, uint32_t bin_size, uint32_t cap,
                         int64_t* cand_off, int32_t* cand_bin, uint64_t* n_cand_out, void* hip_stream) {
  clear_error();
  if (!csd || !rd || !n_cand_out) return set_error(GRIM_EINVAL, "NULL argument");
  if (bin_size == 0) return set_error(GRIM_EINVAL, "bin_size must be >= 1");
  if (cap == 0) return set_error(GRIM_EINVAL, "cap must be >= 1");
  if (!cand_off || (rd->n_reads && !cand_bin)) return set_error(GRIM_EINVAL, "cand_off / cand_bin is NULL");
  if (rd->n_reads && !rd->offsets) return set_error(GRIM_EINVAL, "reads.offsets is NULL");
  if (rd->n_bases && !rd->bases) return set_error(GRIM_EINVAL, "reads.bases is NULL");
  grim_seeds* sd = const_cast<grim_seeds*>(csd);
  std::lock_guard<std::mutex> lk(sd->mu);
  SeedGuard g(sd->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const uint64_t n = rd->n_reads;
  if (!sd->total_host) GRIM_HIP_TRY(hipHostMalloc(&sd->total_host, 4 * sizeof(uint64_t), hipHostMallocDefault));
  *n_cand_out = 0;
  if (n == 0) {
    sd->total_host[0] = 0;
    GRIM_HIP_TRY(hipMemcpyAsync(cand_off, sd->total_host, sizeof(int64_t), hipMemcpyHostToDevice, s));
    GRIM_HIP_TRY(hipStreamSynchronize(s));
    return GRIM_OK;
  }
  // reads on the device
  const uint8_t* bases = rd->bases;
  const int64_t* offsets = rd->offsets;
  if (!rd->on_device) {
    const uint64_t ob = (rd->n_bases + 255) / 256 * 256;
    int rc = grow_dev(&sd->staging, &sd->staging_cap, ob + (n + 1) * 8);
    if (rc) return rc;
    if (rd->n_bases) GRIM_HIP_TRY(hipMemcpyAsync(sd->staging, rd->bases, rd->n_bases, hipMemcpyHostToDevice, s));
    GRIM_HIP_TRY(hipMemcpyAsync(sd->staging + ob, rd->offsets, (n + 1) * 8, hipMemcpyHostToDevice, s));
    bases = sd->staging;
    offsets = reinterpret_cast<const int64_t*>(sd->staging + ob);
  }
  // 1. hits per read
  int rc = grow_dev(&sd->hits, &sd->hits_cap, n);
  if (rc) return rc;
  if (sd->hits_host_cap < n || !sd->hits_host) {
    if (sd->hits_host) (void)hipHostFree(sd->hits_host);
    sd->hits_host = nullptr;
    sd->hits_host_cap = 0;
    GRIM_HIP_TRY(hipHostMalloc(&sd->hits_host, sd->hits_cap * sizeof(uint64_t), hipHostMallocDefault));
    sd->hits_host_cap = sd->hits_cap;
  }
  if (!sd->words) GRIM_HIP_TRY(hipMalloc(&sd->words, 8 * sizeof(uint64_t)));
  uint32_t* bad = reinterpret_cast<uint32_t*>(sd->words + 2);
  uint32_t* n_redo = reinterpret_cast<uint32_t*>(sd->words + 3);
  GRIM_HIP_TRY(launch_zero_words(reinterpret_cast<uint32_t*>(sd->words), 16, s));  // base, bad, n_redo
  hipLaunchKernelGGL(k_seed_hits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sd->start, sd->k, bases,
                     rd->n_bases, offsets, n, sd->hits, bad);
  GRIM_HIP_TRY(hipGetLastError());
  GRIM_HIP_TRY(hipMemcpyAsync(sd->hits_host, sd->hits, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  uint32_t* bad_host = reinterpret_cast<uint32_t*>(sd->total_host + 3);
  GRIM_HIP_TRY(hipMemcpyAsync(bad_host, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  if (*bad_host) return set_error(GRIM_EINVAL, "read offsets out of order or outside [0, n_bases]");
  const uint64_t* H = sd->hits_host;
  // bins lie in [0, nbins): max(p - o, 0) / B <= (G - 1) / B
  const uint64_t max_bin = sd->G / bin_size;
  if (max_bin > 0x7FFFFFFFull) return set_error(GRIM_EINVAL, "more than 2^31 bins");
  const uint32_t nbins = (uint32_t)(max_bin + 1);
  const uint32_t key_bits = 32u - (uint32_t)__builtin_clz(nbins);  // the all-ones key is no bin
  uint32_t vb = 32u - key_bits;
  if (const char* e = std::getenv("GRIM_SEED_VOTE_BITS")) vb = std::min<uint32_t>(vb, (uint32_t)std::max(1, std::atoi(e)));
  const bool all_fallback = vb < 2 || env_flag("GRIM_SEED_FALLBACK_ALL");
  const uint32_t class_min = (uint32_t)std::min((int)kSeedClasses - 1, std::max(0, env_int("GRIM_SEED_CLASS_MIN", 0)));
  SelArgs a{};
  a.start = sd->start;
  a.pos = sd->pos;
  a.k = sd->k;
  a.bases = bases;
  a.offsets = offsets;
  a.hits = sd->hits;
  a.cap = cap;
  a.nbins = nbins;
  a.bin_bits = nbins <= 1 ? 1u : 32u - (uint32_t)__builtin_clz(nbins - 1);
  a.vb = vb;
  make_div(bin_size, &a.dm, &a.ds1, &a.ds2);
  a.range_hits = (uint32_t)std::max(1, env_int("GRIM_SEED_RANGE_HITS", 16384));
  a.force_ranges = env_flag("GRIM_SEED_FORCE_RANGES") ? 1u : 0u;
  a.n_redo = n_redo;
  // 2. batches of bounded staging (each read takes min(hits, cap) slots),
  // planned before anything is launched: every buffer is then allocated
  // once, each batch's host arrays have a region of their own, and batches
  // follow each other on the stream with no host wait in between (the host
  // prepares batch b + 1 while the device runs batch b)
  const uint64_t limit = batch_keys();
  struct Batch {
    uint64_t r0, r1, slots, max_h;
  };
  std::vector<Batch> plan;
  uint64_t nb_max = 0, slots_max = 1, max_h_all = 0;
  for (uint64_t r0 = 0; r0 < n;) {
    uint64_t r1 = r0, slots = 0, max_h = 0;
    while (r1 < n && (r1 == r0 || (slots + std::min<uint64_t>(H[r1], cap) <= limit && r1 - r0 < (1ull << 26)))) {
      if (H[r1] > 0xFFFFFFFFull - 64)
        return set_error(GRIM_ENOMEM, "seed hits of read %llu exceed 2^32", (unsigned long long)r1);
      slots += std::min<uint64_t>(H[r1], cap);
      max_h = std::max(max_h, H[r1]);
      ++r1;
    }
    plan.push_back({r0, r1, slots, max_h});
    nb_max = std::max(nb_max, r1 - r0);
    slots_max = std::max(slots_max, slots);
    max_h_all = std::max(max_h_all, max_h);
    r0 = r1;
  }
  if (sd->host_cap < n) {
    if (sd->toff_host) (void)hipHostFree(sd->toff_host);
    if (sd->list_host) (void)hipHostFree(sd->list_host);
    sd->toff_host = nullptr;
    sd->list_host = nullptr;
    sd->host_cap = 0;
    const uint64_t c = n + n / 8 + 64;
    GRIM_HIP_TRY(hipHostMalloc(&sd->toff_host, c * sizeof(uint64_t), hipHostMallocDefault));
    GRIM_HIP_TRY(hipHostMalloc(&sd->list_host, c * sizeof(uint32_t), hipHostMallocDefault));
    sd->host_cap = c;
  }
  const uint64_t np2 = max_h_all <= 1 ? 1 : 1ull << (64 - __builtin_clzll(max_h_all - 1));
  const uint64_t slab_words = np2 + 2 * max_h_all + 64;
  const uint64_t fb_waves = std::max<uint64_t>(1, std::min<uint64_t>(512, (128ull << 20) / (slab_words * 4)));
  if ((rc = grow_dev(&sd->tmp, &sd->tmp_cap, slots_max))) return rc;
  if ((rc = grow_dev(&sd->toff, &sd->toff_cap, nb_max))) return rc;
  if ((rc = grow_dev(&sd->outoff, &sd->outoff_cap, nb_max))) return rc;
  if ((rc = grow_dev(&sd->bsum, &sd->bsum_cap, scan_blocks(nb_max) + 1))) return rc;
  if ((rc = grow_dev(&sd->cnt, &sd->cnt_cap, nb_max))) return rc;
  if ((rc = grow_dev(&sd->list, &sd->list_cap, nb_max))) return rc;
  if ((rc = grow_dev(&sd->redo, &sd->redo_cap, nb_max))) return rc;
  if ((rc = grow_dev(&sd->slab, &sd->slab_cap, slab_words * fb_waves))) return rc;
  uint64_t nbatch = 0;
  for (const Batch& bt : plan) {
    const uint64_t r0 = bt.r0, nb = bt.r1 - bt.r0;
    // host side, in this batch's region: staging offsets and the reads of
    // each launch, grouped by table size
    uint64_t* toff_h = sd->toff_host + r0;
    uint32_t* list_h = sd->list_host + r0;
    uint64_t per_class[kSeedClasses] = {}, n_fb = 0;
    uint64_t run = 0;
    for (uint64_t i = 0; i < nb; ++i) {
      const uint64_t h = H[r0 + i];
      toff_h[i] = run;
      run += std::min<uint64_t>(h, cap);
      if (h == 0) continue;
      if (all_fallback) {
        ++n_fb;
        continue;
      }
      ++per_class[std::max(class_min, seed_class(h))];
    }
    uint64_t first[kSeedClasses + 1] = {};
    for (uint32_t c = 0; c < kSeedClasses; ++c) first[c + 1] = first[c] + per_class[c];
    {
      uint64_t at[kSeedClasses];
      for (uint32_t c = 0; c < kSeedClasses; ++c) at[c] = first[c];
      uint64_t fb = 0;
      for (uint64_t i = 0; i < nb; ++i) {
        const uint64_t h = H[r0 + i];
        if (h == 0) continue;
        if (all_fallback) list_h[fb++] = (uint32_t)i;
        else list_h[at[std::max(class_min, seed_class(h))]++] = (uint32_t)i;
      }
    }
    const uint64_t listed = all_fallback ? n_fb : first[kSeedClasses];
    GRIM_HIP_TRY(hipMemcpyAsync(sd->toff, toff_h, nb * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    GRIM_HIP_TRY(launch_zero_words(sd->cnt, (uint32_t)nb, s));
    if (listed) GRIM_HIP_TRY(hipMemcpyAsync(all_fallback ? sd->redo : sd->list, list_h, listed * sizeof(uint32_t),
                                            hipMemcpyHostToDevice, s));
    GRIM_HIP_TRY(launch_fill_word(n_redo, all_fallback ? (uint32_t)n_fb : 0u, s));
    a.r0 = r0;
    a.tmp_off = sd->toff;
    a.tmp = sd->tmp;
    a.cnt = sd->cnt;
    a.redo = sd->redo;
    // 3. each read's kept bins, in LDS, one workgroup per read
    if (!all_fallback) {
      for (uint32_t c = 0; c < kSeedClasses; ++c) {
        if (!per_class[c]) continue;
        SelArgs b = a;
        b.list = sd->list + first[c];
        b.n_list = (uint32_t)per_class[c];
        const dim3 grid((unsigned)std::min<uint64_t>(per_class[c], 1u << 30));
        switch (c) {
          case 0: hipLaunchKernelGGL((k_seed_select<64, 1024>), grid, dim3(64), 0, s, b); break;
          case 1: hipLaunchKernelGGL((k_seed_select<128, 2048>), grid, dim3(128), 0, s, b); break;
          case 2: hipLaunchKernelGGL((k_seed_select<256, 4096>), grid, dim3(256), 0, s, b); break;
          case 3: hipLaunchKernelGGL((k_seed_select<256, 8192>), grid, dim3(256), 0, s, b); break;
          case 4: hipLaunchKernelGGL((k_seed_select<512, 16384>), grid, dim3(512), 0, s, b); break;
          default: hipLaunchKernelGGL((k_seed_select<1024, 32768>), grid, dim3(1024), 0, s, b); break;
        }
        GRIM_HIP_TRY(hipGetLastError());
      }
    }
    // 4. reads the tables could not take (a wavefront each, in device memory)
    hipLaunchKernelGGL(k_seed_fallback, dim3((unsigned)fb_waves), dim3(64), 0, s, a, sd->slab, slab_words);
    GRIM_HIP_TRY(hipGetLastError());
    // 5. CSR offsets (continuing the previous batches' total) and the lists in place
    uint64_t* base_in = sd->words + (nbatch & 1);
    uint64_t* base_out = sd->words + ((nbatch + 1) & 1);
    GRIM_HIP_TRY(launch_scan(sd->cnt, nb, sd->outoff, sd->bsum, base_in, base_out, s));
    hipLaunchKernelGGL(k_seed_place, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, sd->toff, sd->tmp, sd->cnt,
                       sd->outoff, nb, r0, cand_off, cand_bin);
    GRIM_HIP_TRY(hipGetLastError());
    ++nbatch;
  }
  GRIM_HIP_TRY(hipMemcpyAsync(sd->total_host + 2, sd->words + (nbatch & 1), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  GRIM_HIP_TRY(hipMemcpyAsync(cand_off + n, sd->total_host + 2, sizeof(int64_t), hipMemcpyHostToDevice, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  *n_cand_out = sd->total_host[2];
  return GRIM_OK;
}

int grim_reverse_complement(const uint8_t* bases, uint64_t n_bases, const int64_t* offsets, uint64_t n_reads,
                            uint8_t* out, void* hip_stream) {
  clear_error();
  if (n_reads == 0) return GRIM_OK;
  if (!offsets || !out || (n_bases && !bases)) return set_error(GRIM_EINVAL, "NULL argument");
  if (n_reads > (1ull << 36)) return set_error(GRIM_EINVAL, "too many reads");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  uint32_t* bad = nullptr;  // set by the kernel when a read's offsets are out of order or out of range
  GRIM_HIP_TRY(hipMalloc(&bad, sizeof(uint32_t)));
  uint32_t bad_host = 0;
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(uint32_t), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_revcomp, dim3((unsigned)((n_reads + 3) / 4)), dim3(256), 0, s, bases, n_bases, offsets,
                       n_reads, out, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad_host, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(bad);
  GRIM_HIP_TRY(e);
  if (bad_host) return set_error(GRIM_EINVAL, "offsets out of order or outside [0, n_bases]; those reads were not written");
  return GRIM_OK;
}

}  // extern "C"
