// Launch order of the all-bins scan: reads sorted by their number of
// 32-token blocks, longest first. The reads that share a wavefront then run
// the same number of loop iterations even when lengths are mixed (100, 150
// and 250 bp reads in one batch), and the longest work starts first. The
// order changes no result: every read's mask row is computed independently.
//
// Two-level counting sort over 64 buckets: each workgroup histograms a
// contiguous range of reads, one workgroup turns the per-range histograms
// into per-range output bases, and each workgroup scatters its range with
// LDS-local cursors. No global atomics, and reads keep (nearly) their input
// order inside a bucket, so a read chunk still touches contiguous tokens.

#include <algorithm>

#include "grim_internal.h"

namespace grim {
namespace {

constexpr uint32_t kBuckets = 64;
constexpr uint32_t kMaxRanges = 1024;  // workgroups of the histogram and scatter passes

__device__ __forceinline__ uint32_t bucket_of(const int64_t* offsets, uint64_t r, uint32_t q) {
  const int64_t L = offsets[r + 1] - offsets[r];
  const uint64_t ntok = L >= (int64_t)q ? (uint64_t)(L - q + 1) : 0;
  const uint64_t nblk = (ntok + 31) >> 5;
  return kBuckets - 1 - (uint32_t)(nblk < kBuckets - 1 ? nblk : kBuckets - 1);
}

__device__ __forceinline__ void range_of(uint64_t n, uint32_t k, uint64_t* lo, uint64_t* hi) {
  const uint64_t per = (n + kMaxRanges - 1) / kMaxRanges;
  *lo = min(n, (uint64_t)k * per);
  *hi = min(n, *lo + per);
}

// hist[k][b]: reads of range k in bucket b
__global__ __launch_bounds__(256) void k_order_hist(const int64_t* offsets, uint64_t n, uint32_t q,
                                                   const DynSizes* dyn, uint32_t* hist) {
  __shared__ uint32_t h[kBuckets];
  if (threadIdx.x < kBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t nn = dyn ? min(dyn->n_reads, n) : n;
  uint64_t lo, hi;
  range_of(nn, blockIdx.x, &lo, &hi);
  for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) atomicAdd(&h[bucket_of(offsets, r, q)], 1u);
  __syncthreads();
  if (threadIdx.x < kBuckets) hist[blockIdx.x * kBuckets + threadIdx.x] = h[threadIdx.x];
}

// hist[k][b] <- first output position of range k's reads in bucket b
__global__ __launch_bounds__(kBuckets) void k_order_prefix(uint32_t* hist) {
  __shared__ uint32_t total[kBuckets];
  const uint32_t b = threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t k = 0; k < kMaxRanges; ++k) {
    const uint32_t c = hist[k * kBuckets + b];
    hist[k * kBuckets + b] = acc;
    acc += c;
  }
  total[b] = acc;
  __syncthreads();
  uint32_t base = 0;
  for (uint32_t i = 0; i < b; ++i) base += total[i];
  for (uint32_t k = 0; k < kMaxRanges; ++k) hist[k * kBuckets + b] += base;
}

__global__ __launch_bounds__(256) void k_order_scatter(const int64_t* offsets, uint64_t n, uint32_t q,
                                                      const DynSizes* dyn, const uint32_t* hist, uint32_t* order) {
  __shared__ uint32_t cur[kBuckets];
  if (threadIdx.x < kBuckets) cur[threadIdx.x] = hist[blockIdx.x * kBuckets + threadIdx.x];
  __syncthreads();
  const uint64_t nn = dyn ? min(dyn->n_reads, n) : n;
  uint64_t lo, hi;
  range_of(nn, blockIdx.x, &lo, &hi);
  for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x)
    order[atomicAdd(&cur[bucket_of(offsets, r, q)], 1u)] = (uint32_t)r;
}

}  // namespace

uint64_t length_order_scratch_words() { return (uint64_t)kMaxRanges * kBuckets; }

hipError_t launch_length_order(const int64_t* offsets, uint64_t n, uint32_t q, const DynSizes* dyn, uint32_t* hist,
                               uint32_t* order, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_hist, dim3(kMaxRanges), dim3(256), 0, s, offsets, n, q, dyn, hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_prefix, dim3(1), dim3(kBuckets), 0, s, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_order_scatter, dim3(kMaxRanges), dim3(256), 0, s, offsets, n, q, dyn, hist, order);
  return hipGetLastError();
}

}  // namespace grim
