// Microbenchmarks behind the all-bins scan's ceilings on gfx950.
//
// 1. VALU issue: independent v_bitop3 chains in registers, 4 and 8 waves per
//    SIMD. A SIMD issues up to two wave64 VALU instructions per 4 cycles (from
//    two waves), so the rate approaches 2 per 4-cycle slot.
// 2. LDS reads: 16-byte ds_read_b128 per lane from a 64 KB array by 16 waves
//    per CU, 8-lane groups each reading one 128-byte row (the scan's layout):
//    rows at random, and rows whose parity alternates between the two groups
//    of a 16-lane bank pass.
// 3. Mix: one such conflict-free ds_read_b128 per step plus K independent
//    bitop3 and the 4 xors that consume the read, 16 waves per CU: the
//    CU-cycles per wavefront step for the instruction mix of the scan's loop
//    (about 10 VALU instructions per 16-byte read per lane).
//
// Every LDS address is masked into the array; every value read feeds the
// output, so no load is dropped. Cycles are priced at 2.4 GHz.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);          \
      std::exit(1);                                                                        \
    }                                                                                      \
  } while (0)

constexpr double kClock = 2.4e9;
constexpr int kCUs = 256;

// ---- 1. VALU issue ----------------------------------------------------------
__global__ __launch_bounds__(256) void k_valu(uint32_t* out, int iters, uint32_t seed) {
  uint32_t a[16];
  for (int i = 0; i < 16; ++i) a[i] = seed * (threadIdx.x + 7 * i);
  const uint32_t k = seed | 1u, m = seed ^ 0x5555u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(a[i]) : "v"(a[i]), "v"(k), "v"(m));
  }
  uint32_t s = 0;
  for (int i = 0; i < 16; ++i) s += a[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// rows for 8-lane group g: MODE 0 at random, MODE 1 with the parity of g
template <int MODE>
__device__ __forceinline__ void row_addresses(uint32_t (&ad)[16], uint32_t seed) {
  const uint32_t lane = threadIdx.x & 63u, g = lane >> 3, s = lane & 7u;
  uint32_t x = seed * (threadIdx.x / 64 + 1) + blockIdx.x * 977u;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    x = x * 1664525u + 1013904223u;
    const uint32_t h = (x ^ (g * 0x9E3779B9u)) * 2246822519u;
    uint32_t row = (h >> 16) & 511u;
    if (MODE == 1) row = (row & ~1u) | (g & 1u);
    ad[u] = (row * 128u + s * 16u) & 0xFFF0u;
  }
}

// ---- 2. LDS reads -------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(1024) void k_lds(uint32_t* out, int iters, uint32_t seed) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[16384];
  for (uint32_t i = threadIdx.x; i < 16384; i += blockDim.x) lds[i] = i * 2654435761u + seed;
  __syncthreads();
  uint32_t ad[16];
  row_addresses<MODE>(ad, seed);
  uint32_t acc0 = 0, acc1 = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      asm volatile("" : "+v"(ad[u]));  // keeps the read inside the loop
      const uint4 v = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(lds) + ad[u]);
      acc0 = __builtin_amdgcn_bitop3_b32(acc0, v.x, v.y, 0x96);
      acc1 = __builtin_amdgcn_bitop3_b32(acc1, v.z, v.w, 0x96);
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc0 + acc1;
}

// ---- 3. LDS + VALU mix --------------------------------------------------------
template <int K>
__global__ __launch_bounds__(1024) void k_mix(uint32_t* out, int iters, uint32_t seed) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[16384];
  for (uint32_t i = threadIdx.x; i < 16384; i += blockDim.x) lds[i] = i * 2654435761u + seed;
  __syncthreads();
  uint32_t ad[16];
  row_addresses<1>(ad, seed);
  uint32_t acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = seed + i * threadIdx.x;
  const uint32_t k1 = seed | 1u, k2 = seed ^ 0x3333u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      asm volatile("" : "+v"(ad[u]));
      const uint4 v = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(lds) + ad[u]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = (u * K + k) & 15;
        asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(acc[i]) : "v"(acc[i]), "v"(k1), "v"(k2));
      }
      acc[u] ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) r += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

template <typename F>
float time_ms(F f) {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  f();
  CK(hipGetLastError());
  CK(hipEventRecord(e0));
  for (int r = 0; r < 5; ++r) f();
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0;
  CK(hipEventElapsedTime(&ms, e0, e1));
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return ms / 5;
}

template <int K>
void mix(uint32_t* out) {
  const int iters = 1000;
  const double steps_per_cu = 16.0 * iters * 16;  // 16 waves per CU, 16 steps per iteration
  const float ms = time_ms([&] { hipLaunchKernelGGL(k_mix<K>, dim3(kCUs), dim3(1024), 0, 0, out, iters, 3u); });
  const double cyc = ms * 1e-3 * kClock / steps_per_cu;
  std::printf("mix  %2d VALU per 16-byte read: %.2f CU-cycles per wavefront step, %.0f B/clk/CU of LDS\n", K + 4, cyc,
              1024.0 / cyc);
}

int main() {
  uint32_t* out;
  CK(hipMalloc(&out, (size_t)kCUs * 8 * 256 * 4));
  for (int wps : {4, 8}) {
    const int blocks = kCUs * wps, iters = 2000;
    const double insts = (double)blocks * 4 * iters * 128;
    const float ms = time_ms([&] { hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(256), 0, 0, out, iters, 3u); });
    const double slots = kCUs * 4 * kClock * ms * 1e-3 / 4;
    std::printf("valu %d waves per SIMD: %.2f VALU instructions per 4-cycle slot per SIMD\n", wps, insts / slots);
  }
  {
    const int iters = 2000;
    const double bytes = (double)kCUs * 1024 * iters * 16 * 16;
    const float m0 = time_ms([&] { hipLaunchKernelGGL(k_lds<0>, dim3(kCUs), dim3(1024), 0, 0, out, iters, 3u); });
    const float m1 = time_ms([&] { hipLaunchKernelGGL(k_lds<1>, dim3(kCUs), dim3(1024), 0, 0, out, iters, 3u); });
    std::printf("lds  random 128-byte rows: %.0f B/clk/CU\n", bytes / (m0 * 1e-3) / kCUs / kClock);
    std::printf("lds  rows of opposite parity per bank pass: %.0f B/clk/CU\n", bytes / (m1 * 1e-3) / kCUs / kClock);
  }
  mix<0>(out);
  mix<2>(out);
  mix<4>(out);
  mix<5>(out);
  mix<6>(out);
  mix<8>(out);
  mix<12>(out);
  CK(hipFree(out));
  return 0;
}
