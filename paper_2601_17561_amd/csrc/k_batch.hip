// Grouped element kernels of the batched CCMM: one persistent launch lifts and digit-splits the
// query columns of every problem of a batch, another rescales every problem's output.  Each
// reads its work list from a device-resident descriptor table, so the same launches (and a
// hipGraph that captured them) serve any batch that fits the workspace: the host only rewrites
// the table.  Work is dealt in chunks of 256 elements; every problem starts at a multiple of
// 256, so one chunk never straddles two problems.
#include "hfe_device.h"

namespace hfe {

constexpr int kChunk = 256;

// The problem a chunk starting at element e belongs to.  e is uniform over the block, so the
// result is too; readfirstlane lets the compiler read the problem's descriptor with scalar loads.
__device__ __forceinline__ int find_problem(const int64_t* begins, int n, int64_t e) {
  int lo = 0, hi = n - 1;  // last problem whose first element is <= e
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begins[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

__global__ void __launch_bounds__(kChunk) k_lift_batched(const BatchElemHeader* hdr, const BatchLiftDesc* d,
                                                         int64_t K, int64_t KB) {
  __shared__ int64_t begins[kMaxBatch];
  const int n = hdr->n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) begins[i] = d[i].elem_begin;
  __syncthreads();
  const int64_t total = hdr->total, kpad = KB * kKB;
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < total; base += (int64_t)gridDim.x * kChunk) {
    const int b = find_problem(begins, n, base);
    const BatchLiftDesc& p = d[b];
    const int64_t e = base + threadIdx.x - p.elem_begin;
    if (e >= p.d3_pad * kpad) continue;
    lift_element(p.XT, p.d3, K, KB, p.d3_pad, p.la, nullptr, p.Xd, e / kpad, e % kpad);
  }
}

__global__ void __launch_bounds__(kChunk) k_rescale_batched(const BatchElemHeader* hdr, const BatchRescaleDesc* d) {
  __shared__ int64_t begins[kMaxBatch];
  const int n = hdr->n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) begins[i] = d[i].elem_begin;
  __syncthreads();
  const int64_t total = hdr->total;
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < total; base += (int64_t)gridDim.x * kChunk) {
    const int b = find_problem(begins, n, base);
    const BatchRescaleDesc& p = d[b];
    const int64_t e = base + threadIdx.x - p.elem_begin;
    if (e >= p.n) continue;
    rescale_element(p.C, p.C + (int64_t)p.ra.level * p.n, p.n, p.ra, p.out, e);
  }
}

hipError_t launch_lift_batched(const BatchElemHeader* hdr, const BatchLiftDesc* d, int64_t K, int64_t KB,
                               int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_lift_batched, dim3((unsigned)grid), dim3(kChunk), 0, s, hdr, d, K, KB);
  return hipGetLastError();
}

hipError_t launch_rescale_batched(const BatchElemHeader* hdr, const BatchRescaleDesc* d, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_rescale_batched, dim3((unsigned)grid), dim3(kChunk), 0, s, hdr, d);
  return hipGetLastError();
}

}  // namespace hfe
