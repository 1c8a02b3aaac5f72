// Launch order of the all-bins scan: reads sorted by their number of
// 32-token blocks, longest first. The reads that share a wavefront then run
// the same number of loop iterations even when lengths are mixed (100, 150
// and 250 bp reads in one batch), and the longest work starts first. The
// order changes no result: every read's mask row is computed independently.
//
// Within a length class, reads with even and odd indices alternate: launch
// position k holds a read whose index has the parity of k, as far as the two
// parities last. The scan's token lists are ordered by the parity of each
// token's row with the opposite preference for even and odd reads (see the
// tokenizer), and reads at launch positions 2p and 2p+1 share a bank pass of
// the scan's LDS reads: at most token positions one of them reads a row of
// even index and the other one of odd index, which fall in different halves
// of the LDS banks.
//
// Two-level counting sort over 64 length classes x 2 parities: each
// workgroup histograms a contiguous range of reads, one workgroup turns the
// per-range histograms into per-range starting indices and per-class bases,
// and each workgroup scatters its range with LDS-local cursors. No global
// atomics.

#include <algorithm>

#include "grim_internal.h"

namespace grim {
namespace {

constexpr uint32_t kBuckets = 64;                 // length classes
constexpr uint32_t kKeys = 2 * kBuckets;          // (class, read-index parity)
constexpr uint32_t kMaxRanges = 1024;             // workgroups of the histogram and scatter passes

__device__ __forceinline__ uint32_t bucket_of(const int64_t* offsets, uint64_t r, uint32_t q) {
  const int64_t L = offsets[r + 1] - offsets[r];
  const uint64_t ntok = L >= (int64_t)q ? (uint64_t)(L - q + 1) : 0;
  const uint64_t nblk = (ntok + 31) >> 5;
  return kBuckets - 1 - (uint32_t)(nblk < kBuckets - 1 ? nblk : kBuckets - 1);
}

__device__ __forceinline__ uint32_t key_of(const int64_t* offsets, uint64_t r, uint32_t q) {
  return 2u * bucket_of(offsets, r, q) + (uint32_t)(r & 1u);
}

__device__ __forceinline__ void range_of(uint64_t n, uint32_t k, uint64_t* lo, uint64_t* hi) {
  const uint64_t per = (n + kMaxRanges - 1) / kMaxRanges;
  *lo = min(n, (uint64_t)k * per);
  *hi = min(n, *lo + per);
}

// hist[k][key]: reads of range k with that key
__global__ __launch_bounds__(256) void k_order_hist(const int64_t* offsets, uint64_t n, uint32_t q,
                                                   const DynSizes* dyn, uint32_t* hist) {
  __shared__ uint32_t h[kKeys];
  if (threadIdx.x < kKeys) h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t nn = dyn ? min(dyn->n_reads, n) : n;
  uint64_t lo, hi;
  range_of(nn, blockIdx.x, &lo, &hi);
  for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) atomicAdd(&h[key_of(offsets, r, q)], 1u);
  __syncthreads();
  if (threadIdx.x < kKeys) hist[blockIdx.x * kKeys + threadIdx.x] = h[threadIdx.x];
}

// hist[k][key] <- index, among the reads with that key, of range k's first
// one; tab[2c] <- first launch position of class c, tab[2c + 1] <- the
// number of read pairs that alternate in it (the smaller parity count)
__global__ __launch_bounds__(kKeys) void k_order_prefix(uint32_t* hist) {
  __shared__ uint32_t total[kKeys];
  const uint32_t key = threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t k = 0; k < kMaxRanges; ++k) {
    const uint32_t c = hist[k * kKeys + key];
    hist[k * kKeys + key] = acc;
    acc += c;
  }
  total[key] = acc;
  __syncthreads();
  if (key < kBuckets) {
    uint32_t base = 0;
    for (uint32_t c = 0; c < key; ++c) base += total[2 * c] + total[2 * c + 1];
    uint32_t* tab = hist + kMaxRanges * kKeys;
    tab[2 * key] = base;
    tab[2 * key + 1] = min(total[2 * key], total[2 * key + 1]);
  }
}

__global__ __launch_bounds__(256) void k_order_scatter(const int64_t* offsets, uint64_t n, uint32_t q,
                                                      const DynSizes* dyn, const uint32_t* hist, uint32_t* order) {
  __shared__ uint32_t cur[kKeys];
  if (threadIdx.x < kKeys) cur[threadIdx.x] = hist[blockIdx.x * kKeys + threadIdx.x];
  __syncthreads();
  const uint32_t* tab = hist + kMaxRanges * kKeys;
  const uint64_t nn = dyn ? min(dyn->n_reads, n) : n;
  uint64_t lo, hi;
  range_of(nn, blockIdx.x, &lo, &hi);
  for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) {
    const uint32_t key = key_of(offsets, r, q), c = key >> 1, f = key & 1u;
    const uint32_t i = atomicAdd(&cur[key], 1u);
    const uint32_t base = tab[2 * c], m = tab[2 * c + 1];
    // the first m reads of each parity alternate (position parity = read
    // parity); the rest of the larger parity follow them
    const uint32_t pos = i < m ? base + 2u * i + (f ^ (base & 1u)) : base + 2u * m + (i - m);
    order[pos] = (uint32_t)r;
  }
}

}  // namespace

uint64_t length_order_scratch_words() { return (uint64_t)kMaxRanges * kKeys + 2 * kBuckets; }

hipError_t launch_length_order(const int64_t* offsets, uint64_t n, uint32_t q, const DynSizes* dyn, uint32_t* hist,
                               uint32_t* order, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_hist, dim3(kMaxRanges), dim3(256), 0, s, offsets, n, q, dyn, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_prefix, dim3(1), dim3(kKeys), 0, s, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_scatter, dim3(kMaxRanges), dim3(256), 0, s, offsets, n, q, dyn, hist, order);
  return hipGetLastError();
}

}  // namespace grim
