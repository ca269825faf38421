// Rate probes: the instruction rates that bound the two contraction forms, measured on the device
// the library runs on, so that each form's achieved rate can be set against a measured ceiling
// beside the published peak.
//
//  * int8 MFMA (v_mfma_i32_32x32x32_i8), operands streaming: every wave rotates through a pool of
//    eight query-like and eight database-like operand registers holding random bytes and
//    re-randomises two of them (xorshift) between groups of 16 products, so consecutive products
//    see new random bits, as the contraction's digit planes do.  The chip's clock under that
//    switching load, not instruction issue, sets this ceiling.
//  * the same with all-zero operands: the issue ceiling at the clock the chip holds when the
//    operands do not switch.
//  * VALU 32 x 32 -> 64-bit multiply-add (v_mad_u64_u32), the instruction the plain form spends
//    four of per residue multiply-add: eight independent chains per lane.
#include "hfe_device.h"

namespace hfe {

__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
  // 32-bit integer finaliser (an avalanche mix), used only to fill operands with random bits
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ v4i xorshift4(v4i v) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t x = (uint32_t)v[i];
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    v[i] = (int)x;
  }
  return v;
}

template <bool kZero>
__global__ void __launch_bounds__(256) k_probe_mfma_i8(int64_t iters, int32_t* sink) {
  const uint32_t id = (blockIdx.x * 256u + threadIdx.x) * 64u;
  v4i a[8], b[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[j][i] = kZero ? 0 : (int)probe_hash(id + 8 * j + i);
      b[j][i] = kZero ? 0 : (int)probe_hash(id + 32 + 8 * j + i);
    }
  v16i acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        acc[j & 3] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[(j + r) & 7], b[(3 * j + r) & 7], acc[j & 3], 0, 0, 0);
      if (!kZero) {
        a[r] = xorshift4(a[r]);
        b[r] = xorshift4(b[r]);
      }
    }
  }
  int32_t x = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int e = 0; e < 16; ++e) x ^= acc[u][e];
  sink[blockIdx.x * 256 + threadIdx.x] = x;
}

__global__ void __launch_bounds__(256) k_probe_mad_u64(int64_t iters, uint64_t* sink) {
  const uint32_t id = blockIdx.x * 256u + threadIdx.x;
  uint64_t acc[8];
  uint32_t y[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    acc[j] = probe_hash(id * 16 + j);
    y[j] = probe_hash(id * 16 + 8 + j) | 1u;
  }
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = (uint64_t)(uint32_t)acc[j] * y[j] + acc[j];
  }
  uint64_t x = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) x ^= acc[j];
  sink[id] = x;
}

// MFMA probes: 128 products of 32 x 32 x 32 per wave per iteration; the VALU probe: 64
// multiply-adds per lane per iteration.
hipError_t launch_probe(int which, int64_t iters, int grid, void* sink, hipStream_t s) {
  if (which == 1)
    hipLaunchKernelGGL(k_probe_mfma_i8<false>, dim3(grid), dim3(256), 0, s, iters, static_cast<int32_t*>(sink));
  else if (which == 2)
    hipLaunchKernelGGL(k_probe_mfma_i8<true>, dim3(grid), dim3(256), 0, s, iters, static_cast<int32_t*>(sink));
  else if (which == 3)
    hipLaunchKernelGGL(k_probe_mad_u64, dim3(grid), dim3(256), 0, s, iters, static_cast<uint64_t*>(sink));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace hfe
