// Per-read summaries of pass masks: the number of passing bins and a 64-bit
// digest of the row, for consumers that keep the masks (189 KB per read at
// human scale) in device memory and copy only these back.
//
// digest = sum over words i of mix64((i << 32) | row[i]) mod 2^64, with mix64
// the SplitMix64 output function (Steele, Lea and Flood 2014). The sum does
// not depend on the order the words are visited in, so any number of threads
// can share a row.
//
// One workgroup per row (grid-stride over rows): the row is read with 16-byte
// loads from its first 16-byte boundary, the few words before and after it
// with 4-byte loads; each thread keeps a popcount and a digest partial, then
// the wavefronts reduce with shuffles and LDS.

#include "grim_internal.h"

namespace grim {
namespace {

constexpr int kSumThreads = 256;
constexpr int kBatch = 4;  // 16-byte loads in flight per thread

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ void add_word(uint64_t i, uint32_t w, uint32_t& pc, uint64_t& dg) {
  pc += (uint32_t)__popc(w);
  dg += mix64((i << 32) | w);
}

__global__ __launch_bounds__(kSumThreads) void k_mask_summary(const uint32_t* mask, uint64_t n, uint64_t W,
                                                              uint32_t* pass_count, uint64_t* digest) {
  __shared__ uint32_t s_pc[kSumThreads / 64];
  __shared__ uint64_t s_dg[kSumThreads / 64];
  const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
  for (uint64_t r = blockIdx.x; r < n; r += gridDim.x) {
    const uint32_t* row = mask + r * W;
    // words before the first 16-byte boundary of the row
    uint64_t head = (4u - ((uint32_t)(reinterpret_cast<uintptr_t>(row) >> 2) & 3u)) & 3u;
    if (head > W) head = W;
    const uint64_t n4 = (W - head) / 4;
    uint32_t pc = 0;
    uint64_t dg = 0;
    if (t < head) add_word(t, row[t], pc, dg);
    const uint4* body = reinterpret_cast<const uint4*>(row + head);
    // kBatch 16-byte loads per thread are issued before any is used, so
    // enough bytes are in flight per CU to cover the memory latency
    uint64_t k = t;
    for (; k + (kBatch - 1) * kSumThreads < n4; k += kBatch * kSumThreads) {
      uint4 v[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) v[b] = body[k + b * kSumThreads];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const uint64_t i = head + 4 * (k + b * kSumThreads);
        add_word(i, v[b].x, pc, dg);
        add_word(i + 1, v[b].y, pc, dg);
        add_word(i + 2, v[b].z, pc, dg);
        add_word(i + 3, v[b].w, pc, dg);
      }
    }
    for (; k < n4; k += kSumThreads) {
      const uint4 v = body[k];
      const uint64_t i = head + 4 * k;
      add_word(i, v.x, pc, dg);
      add_word(i + 1, v.y, pc, dg);
      add_word(i + 2, v.z, pc, dg);
      add_word(i + 3, v.w, pc, dg);
    }
    const uint64_t tail = head + 4 * n4;
    if (tail + t < W) add_word(tail + t, row[tail + t], pc, dg);
    for (int off = 32; off >= 1; off >>= 1) {
      pc += (uint32_t)__shfl_xor((int)pc, off);
      const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)dg, off);
      const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(dg >> 32), off);
      dg += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0) {
      s_pc[wave] = pc;
      s_dg[wave] = dg;
    }
    __syncthreads();
    if (t == 0) {
      uint32_t P = 0;
      uint64_t D = 0;
      for (int w = 0; w < kSumThreads / 64; ++w) {
        P += s_pc[w];
        D += s_dg[w];
      }
      if (pass_count) pass_count[r] = P;
      if (digest) digest[r] = D;
    }
    __syncthreads();  // s_pc / s_dg are reused by the next row
  }
}

}  // namespace
}  // namespace grim

using namespace grim;

extern "C" {

int grim_mask_summary(const uint32_t* mask, uint64_t n_reads, uint64_t mask_words, uint32_t* pass_count_out,
                      uint64_t* digest_out, void* hip_stream) {
  clear_error();
  if (n_reads == 0) return GRIM_OK;
  if (!mask) return set_error(GRIM_EINVAL, "mask is NULL");
  if (mask_words == 0 || mask_words >= (1ull << 32)) return set_error(GRIM_EINVAL, "mask_words must be in [1, 2^32)");
  if (reinterpret_cast<uintptr_t>(mask) & 3u) return set_error(GRIM_EINVAL, "mask is not 4-byte aligned");
  if (n_reads > (1ull << 40) || mask_words > ((1ull << 60) / n_reads))
    return set_error(GRIM_EINVAL, "mask larger than 2^62 bytes");
  if (!pass_count_out && !digest_out) return GRIM_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const uint64_t blocks = n_reads < (1ull << 20) ? n_reads : (1ull << 20);
  hipLaunchKernelGGL(k_mask_summary, dim3((unsigned)blocks), dim3(kSumThreads), 0, s, mask, n_reads, mask_words,
                     pass_count_out, digest_out);
  GRIM_HIP_TRY(hipGetLastError());
  return GRIM_OK;
}

}  // extern "C"
