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
//   2. reads are cut into batches of bounded total hits; per batch
//   3. every hit's bin is written out (a wavefront per read, coalesced reads
//      of each seed's positions), 4. each read's bins are sorted (rocPRIM
//      segmented radix sort on the bin's bits), 5. runs of equal bins become
//      (bin, votes) (a wavefront per read, ballots mark run starts),
//   6. reads with more than `cap` runs find the vote threshold by bisection
//      with wavefront-wide counts, and every read writes its kept bins in bin
//      order into the CSR output.

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

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
  uint32_t* seg = nullptr;        // [batch reads + 1] segment offsets
  uint32_t* cnt = nullptr;        // [batch reads + 1] runs kept per read
  uint32_t* nruns = nullptr;      // [batch reads + 1] runs per read
  uint64_t* outoff = nullptr;     // [batch reads + 1] first output slot (batch-relative)
  uint64_t batch_cap = 0;
  uint32_t* keys_a = nullptr;     // [batch keys] bins, then run start positions
  uint32_t* keys_b = nullptr;     // [batch keys] sorted bins
  uint32_t* runs = nullptr;       // [batch keys] run bins
  uint64_t keys_cap = 0;
  void* tmp = nullptr;            // rocPRIM temporary storage
  size_t tmp_cap = 0;
  uint8_t* staging = nullptr;     // host-resident reads copied in
  uint64_t staging_cap = 0;
  uint64_t* total_host = nullptr; // pinned [4]
  uint32_t* bad = nullptr;        // device word: a read's offsets were rejected
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
__device__ __forceinline__ int64_t seed_code(const uint8_t* s, uint32_t k) {
  uint64_t code = 0;
  for (uint32_t j = 0; j < k; ++j) {
    const int c = base_code(s[j]);
    if (c < 0) return -1;
    code = (code << 2) | (uint64_t)c;
  }
  return (int64_t)code;
}

struct CandArgs2 {
  const uint64_t* start;
  const uint32_t* pos;
  uint32_t k, B, cap;
  const uint8_t* bases;
  const int64_t* offsets;
  uint64_t n_reads;
  uint64_t r0;            // first read of the batch
  uint64_t nb;            // reads in the batch
  const uint32_t* seg;    // [nb + 1] key offsets of the batch's reads
  uint32_t* keys_a;
  uint32_t* keys_b;
  uint32_t* runs;
  uint32_t* cnt;
  uint32_t* nruns;
  const uint64_t* outoff;
  uint64_t out_base;      // output slot of the batch's first candidate
  int64_t* cand_off;
  int32_t* cand_bin;
};

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

__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Every hit's bin, in seed order, into the read's segment of keys_a.
__global__ __launch_bounds__(256) void k_seed_expand(CandArgs2 a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t i = wave_uniform((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (i >= a.nb) return;
  const uint64_t r = a.r0 + i;
  const uint8_t* rd = a.bases + a.offsets[r];
  const int64_t L = a.offsets[r + 1] - a.offsets[r];
  uint64_t w = a.seg[i];
  const int64_t n_seeds = L >= (int64_t)a.k ? L / (int64_t)a.k : 0;
  // up to 64 seeds at a time: lane j codes seed sb + j and looks up its hit
  // range, all in parallel; then the wavefront writes each seed's hits
  for (int64_t sb = 0; sb < n_seeds; sb += 64) {
    uint64_t h0 = 0, h1 = 0;
    if (sb + lane < n_seeds) {
      const int64_t c = seed_code(rd + (sb + lane) * a.k, a.k);
      if (c >= 0) {
        h0 = a.start[c];
        h1 = a.start[c + 1];
      }
    }
    const int64_t m = min<int64_t>(64, n_seeds - sb);
    for (int64_t j = 0; j < m; ++j) {
      const uint64_t H0 = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(h0 >> 32), (int)j) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)h0, (int)j);
      const uint64_t H1 = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(h1 >> 32), (int)j) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)h1, (int)j);
      const int64_t o = (sb + j) * (int64_t)a.k;
      for (uint64_t h = H0 + lane; h < H1; h += 64) {
        const int64_t loc = (int64_t)a.pos[h] - o;
        a.keys_a[w + (h - H0)] = (uint32_t)((loc < 0 ? 0 : loc) / a.B);
      }
      w += H1 - H0;
    }
  }
}

// Runs of equal bins in each sorted segment: run j of read i starts at key
// position keys_a[s0 + j] (overwriting the consumed bins) with bin runs[s0 + j];
// cnt[i] = runs kept (at most cap).
__global__ __launch_bounds__(256) void k_seed_runs(CandArgs2 a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t i = wave_uniform((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (i >= a.nb) return;
  const uint32_t s0 = a.seg[i], s1 = a.seg[i + 1];
  uint32_t nr = 0;
  for (uint32_t c0 = s0; c0 < s1; c0 += 64) {
    const uint32_t idx = c0 + lane;
    const bool valid = idx < s1;
    const uint32_t key = valid ? a.keys_b[idx] : 0u;
    const bool st = valid && (idx == s0 || a.keys_b[idx - 1] != key);
    const uint64_t m = __ballot(st);
    if (st) {
      const uint32_t j = nr + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      a.keys_a[s0 + j] = idx;
      a.runs[s0 + j] = key;
    }
    nr += (uint32_t)__popcll(m);
  }
  if (lane == 0) {
    a.cnt[i] = min(nr, a.cap);
    a.nruns[i] = nr;
  }
}

// Votes of run j of a read whose runs start at rs[0 .. nr) within [.., s1).
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

__global__ __launch_bounds__(256) void k_seed_select(CandArgs2 a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t i = wave_uniform((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  if (i >= a.nb) return;
  const uint64_t r = a.r0 + i;
  const uint32_t s0 = a.seg[i], s1 = a.seg[i + 1];
  const uint64_t out0 = a.out_base + a.outoff[i];
  if (lane == 0) a.cand_off[r] = (int64_t)out0;
  const uint32_t nr = a.nruns[i];  // runs of the read (cnt holds min(runs, cap))
  const uint32_t* rs = a.keys_a + s0;
  const uint32_t* rb = a.runs + s0;
  if (nr <= a.cap) {
    for (uint32_t j = lane; j < nr; j += 64) a.cand_bin[out0 + j] = (int32_t)rb[j];
    return;
  }
  // the largest v with at least cap runs of >= v votes: one pass counts the
  // runs at or above every v up to 32 (votes are few: one per seed); larger
  // thresholds fall back to a bisection
  constexpr uint32_t kHist = 32;
  uint32_t ge[kHist + 1];
#pragma unroll
  for (uint32_t t = 0; t <= kHist; ++t) ge[t] = 0;
  uint32_t vmax = 0;
  for (uint32_t j0 = 0; j0 < nr; j0 += 64) {
    const uint32_t j = j0 + lane;
    const uint32_t v = j < nr ? run_votes(rs, j, nr, s1) : 0u;
    vmax = max(vmax, v);
#pragma unroll
    for (uint32_t t = 1; t <= kHist; ++t) ge[t] += (uint32_t)__popcll(__ballot(v >= t));
  }
  for (int off = 32; off >= 1; off >>= 1) vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off));
  uint32_t lo = 1, hi = vmax;
  if (ge[kHist] < a.cap) {
    // the threshold is at most 32: the largest t with ge[t] >= cap (ge[1] = nr > cap)
    uint32_t vt1 = 1;
#pragma unroll
    for (uint32_t t = 2; t <= kHist; ++t)
      if (ge[t] >= a.cap) vt1 = t;
    lo = hi = vt1;
  } else {
    lo = kHist;
  }
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo + 1) / 2;
    if (count_at_least(rs, nr, s1, mid, lane) >= a.cap) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t vt = lo;
  // runs taken at exactly vt (ge is read with static indexes only, so it stays in registers)
  uint32_t above = 0;
#pragma unroll
  for (uint32_t t = 2; t <= kHist; ++t)
    if (t == vt + 1) above = ge[t];
  const uint32_t need = a.cap - (vt < kHist ? above : count_at_least(rs, nr, s1, vt + 1, lane));
  uint32_t taken = 0, ties = 0;
  for (uint32_t j0 = 0; j0 < nr; j0 += 64) {
    const uint32_t j = j0 + lane;
    const uint32_t v = j < nr ? run_votes(rs, j, nr, s1) : 0;
    const bool tie = j < nr && v == vt;
    const uint64_t tm = __ballot(tie);
    const uint32_t tie_rank = ties + (uint32_t)__popcll(tm & ((1ull << lane) - 1ull));
    const bool keep = j < nr && (v > vt || (tie && tie_rank < need));
    const uint64_t km = __ballot(keep);
    if (keep) a.cand_bin[out0 + taken + (uint32_t)__popcll(km & ((1ull << lane) - 1ull))] = (int32_t)rb[j];
    taken += (uint32_t)__popcll(km);
    ties += (uint32_t)__popcll(tm);
  }
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
  for (void* p : {(void*)sd->start, (void*)sd->pos, (void*)sd->hits, (void*)sd->seg, (void*)sd->cnt,
                  (void*)sd->nruns, (void*)sd->outoff, (void*)sd->keys_a, (void*)sd->keys_b, (void*)sd->runs, sd->tmp,
                  (void*)sd->staging, (void*)sd->bad})
    if (p) (void)hipFree(p);
  if (sd->hits_host) (void)hipHostFree(sd->hits_host);
  if (sd->total_host) (void)hipHostFree(sd->total_host);
  delete sd;
}

// Keys per batch of the candidate passes: 16 bytes of scratch per key
// (GRIM_SEED_BATCH_KEYS overrides, e.g. to exercise many batches in tests).
uint64_t batch_keys() {
  if (const char* e = std::getenv("GRIM_SEED_BATCH_KEYS")) {
    const long long v = std::atoll(e);
    if (v > 0) return (uint64_t)v;
  }
  return 1ull << 29;
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
  size_t tmp_bytes = 0;
  if ((e = rocprim::exclusive_scan(nullptr, tmp_bytes, counts, sd->start, (uint64_t)0, (size_t)(sd->nk + 1),
                                   rocprim::plus<uint64_t>(), s)) != hipSuccess)
    return fail(e, "scan size");
  if ((e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 1))) != hipSuccess) return fail(e, "scan storage");
  if ((e = rocprim::exclusive_scan(tmp, tmp_bytes, counts, sd->start, (uint64_t)0, (size_t)(sd->nk + 1),
                                   rocprim::plus<uint64_t>(), s)) != hipSuccess)
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
  if (!sd->bad) GRIM_HIP_TRY(hipMalloc(&sd->bad, sizeof(uint32_t)));
  GRIM_HIP_TRY(launch_zero_words(sd->bad, 1, s));
  hipLaunchKernelGGL(k_seed_hits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sd->start, sd->k, bases,
                     rd->n_bases, offsets, n, sd->hits, sd->bad);
  GRIM_HIP_TRY(hipGetLastError());
  GRIM_HIP_TRY(hipMemcpyAsync(sd->hits_host, sd->hits, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  uint32_t* bad_host = reinterpret_cast<uint32_t*>(sd->total_host + 3);
  GRIM_HIP_TRY(hipMemcpyAsync(bad_host, sd->bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  if (*bad_host) return set_error(GRIM_EINVAL, "read offsets out of order or outside [0, n_bases]");
  const uint64_t* H = sd->hits_host;
  // largest bin index: max(p - o, 0) / B < G / B
  const uint64_t max_bin = sd->G / bin_size;
  if (max_bin > 0x7FFFFFFFull) return set_error(GRIM_EINVAL, "more than 2^31 bins");
  uint32_t end_bit = 1;
  while (end_bit < 32 && (max_bin >> end_bit)) ++end_bit;
  // 2. batches of bounded total hits
  uint64_t out_base = 0;
  const uint64_t limit = batch_keys();
  std::vector<uint32_t> seg_host;
  for (uint64_t r0 = 0; r0 < n;) {
    uint64_t r1 = r0, keys = 0;
    while (r1 < n && (r1 == r0 || keys + H[r1] <= limit)) keys += H[r1++];
    if (keys > 0xFFFFFFFFull - 64) return set_error(GRIM_ENOMEM, "seed hits of read %llu exceed 2^32", (unsigned long long)r0);
    const uint64_t nb = r1 - r0;
    seg_host.assign(nb + 1, 0);
    for (uint64_t i = 0; i < nb; ++i) seg_host[i + 1] = seg_host[i] + (uint32_t)H[r0 + i];
    if (sd->batch_cap < nb + 1 || !sd->seg) {
      for (void* p : {(void*)sd->seg, (void*)sd->cnt, (void*)sd->nruns, (void*)sd->outoff})
        if (p) (void)hipFree(p);
      sd->seg = nullptr;
      sd->cnt = nullptr;
      sd->nruns = nullptr;
      sd->outoff = nullptr;
      uint64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
      if ((rc = grow_dev(&sd->seg, &c0, nb + 1))) return rc;
      if ((rc = grow_dev(&sd->cnt, &c1, c0))) return rc;
      if ((rc = grow_dev(&sd->nruns, &c3, c0))) return rc;
      if ((rc = grow_dev(&sd->outoff, &c2, c0))) return rc;
      sd->batch_cap = c0;
    }
    uint64_t kc = sd->keys_cap;
    if (sd->keys_cap < keys + 1 || !sd->keys_a) {
      if (sd->keys_a) (void)hipFree(sd->keys_a);
      if (sd->keys_b) (void)hipFree(sd->keys_b);
      if (sd->runs) (void)hipFree(sd->runs);
      sd->keys_a = sd->keys_b = sd->runs = nullptr;
      kc = 0;
      uint64_t c1 = 0, c2 = 0;
      if ((rc = grow_dev(&sd->keys_a, &kc, keys + 1))) return rc;
      if ((rc = grow_dev(&sd->keys_b, &c1, keys + 1))) return rc;
      if ((rc = grow_dev(&sd->runs, &c2, keys + 1))) return rc;
      sd->keys_cap = kc;
    }
    GRIM_HIP_TRY(hipMemcpyAsync(sd->seg, seg_host.data(), (nb + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    CandArgs2 a{};
    a.start = sd->start;
    a.pos = sd->pos;
    a.k = sd->k;
    a.B = bin_size;
    a.cap = cap;
    a.bases = bases;
    a.offsets = offsets;
    a.n_reads = n;
    a.r0 = r0;
    a.nb = nb;
    a.seg = sd->seg;
    a.keys_a = sd->keys_a;
    a.keys_b = sd->keys_b;
    a.runs = sd->runs;
    a.cnt = sd->cnt;
    a.nruns = sd->nruns;
    a.outoff = sd->outoff;
    a.out_base = out_base;
    a.cand_off = cand_off;
    a.cand_bin = cand_bin;
    const unsigned wblocks = (unsigned)((nb + 3) / 4);
    // 3. bins of every hit
    hipLaunchKernelGGL(k_seed_expand, dim3(wblocks), dim3(256), 0, s, a);
    GRIM_HIP_TRY(hipGetLastError());
    // 4. sort each read's bins
    size_t need = 0;
    GRIM_HIP_TRY(rocprim::segmented_radix_sort_keys(nullptr, need, sd->keys_a, sd->keys_b, (unsigned)keys,
                                                    (unsigned)nb, sd->seg, sd->seg + 1, 0u, end_bit, s));
    if (need > sd->tmp_cap || !sd->tmp) {
      if (sd->tmp) (void)hipFree(sd->tmp);
      sd->tmp = nullptr;
      sd->tmp_cap = 0;
      GRIM_HIP_TRY(hipMalloc(&sd->tmp, std::max<size_t>(need, 1)));
      sd->tmp_cap = std::max<size_t>(need, 1);
    }
    size_t have = sd->tmp_cap;
    GRIM_HIP_TRY(rocprim::segmented_radix_sort_keys(sd->tmp, have, sd->keys_a, sd->keys_b, (unsigned)keys,
                                                    (unsigned)nb, sd->seg, sd->seg + 1, 0u, end_bit, s));
    // 5. runs and kept counts
    hipLaunchKernelGGL(k_seed_runs, dim3(wblocks), dim3(256), 0, s, a);
    GRIM_HIP_TRY(hipGetLastError());
    need = 0;
    GRIM_HIP_TRY(rocprim::exclusive_scan(nullptr, need, sd->cnt, sd->outoff, (uint64_t)0, (size_t)nb,
                                         rocprim::plus<uint64_t>(), s));
    if (need > sd->tmp_cap) {
      (void)hipFree(sd->tmp);
      sd->tmp = nullptr;
      sd->tmp_cap = 0;
      GRIM_HIP_TRY(hipMalloc(&sd->tmp, need));
      sd->tmp_cap = need;
    }
    have = sd->tmp_cap;
    GRIM_HIP_TRY(rocprim::exclusive_scan(sd->tmp, have, sd->cnt, sd->outoff, (uint64_t)0, (size_t)nb,
                                         rocprim::plus<uint64_t>(), s));
    // 6. kept bins in bin order
    hipLaunchKernelGGL(k_seed_select, dim3(wblocks), dim3(256), 0, s, a);
    GRIM_HIP_TRY(hipGetLastError());
    // batch total: last offset + last count
    uint32_t last_cnt = 0;
    GRIM_HIP_TRY(hipMemcpyAsync(sd->total_host, sd->outoff + nb - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    GRIM_HIP_TRY(hipMemcpyAsync(sd->total_host + 1, sd->cnt + nb - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    GRIM_HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(&last_cnt, sd->total_host + 1, sizeof last_cnt);
    out_base += sd->total_host[0] + last_cnt;
    r0 = r1;
  }
  sd->total_host[2] = out_base;
  GRIM_HIP_TRY(hipMemcpyAsync(cand_off + n, sd->total_host + 2, sizeof(int64_t), hipMemcpyHostToDevice, s));
  GRIM_HIP_TRY(hipStreamSynchronize(s));
  *n_cand_out = out_base;
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
