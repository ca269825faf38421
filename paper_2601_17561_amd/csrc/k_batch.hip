// Grouped element kernels of the batched CCMM: one persistent launch lifts and splits the query
// columns of every item of a batch (into its problem's planes, at the item's column offset),
// another rescales every item's output, and for the RNS form a third reconstructs every problem's
// residues mod its primes.  Each reads its work list from a device-resident descriptor table, so
// the same launches (and a hipGraph that captured them) serve any batch that fits the workspace:
// the host only rewrites the table.  Work is dealt in chunks of 256 units; every list entry starts
// at a multiple of 256, so one chunk never straddles two entries.
#include "hfe_device.h"

namespace hfe {

constexpr int kChunk = 256;

// The entry a chunk starting at element e belongs to.  e is uniform over the block, so the result
// is too; readfirstlane lets the compiler read the entry's descriptor with scalar loads.
__device__ __forceinline__ int find_problem(const int64_t* begins, int n, int64_t e) {
  int lo = 0, hi = n - 1;  // last entry whose first element is <= e
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begins[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// form 0: 5 digit planes per prime; form n > 0: the RNS form with n small moduli; form -n < 0: the
// n^2 form with n bases (planes M, M' per base).
__global__ void __launch_bounds__(kChunk) k_lift_batched(const BatchElemHeader* hdr, const BatchLiftDesc* d,
                                                         int64_t K, int64_t KB, int form) {
  __shared__ int64_t begins[kMaxBatch];
  const int n = hdr->n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) begins[i] = d[i].elem_begin;
  __syncthreads();
  const int64_t total = hdr->total, kpad = KB * kKB;
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < total; base += (int64_t)gridDim.x * kChunk) {
    const int b = find_problem(begins, n, base);
    const BatchLiftDesc& p = d[b];
    const int64_t e = base + threadIdx.x - p.elem_begin;
    // whole lane quads pass (cols x kpad is a multiple of 4), as the lift's packing needs
    if (e >= p.cols * kpad) continue;
    // columns c >= p.d3 are the problem's padding: lift_residues reports them invalid (zero)
    const int64_t c = e / kpad;
    lift_lane(p.XT, p.d3, K, KB, p.d3_pad, p.la, form, nullptr, p.Xd + p.c0 * kKB, c, e - c * kpad);
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
    const int64_t c = e / p.R_out, r = e - c * p.R_out;
    if (r < p.split)
      rescale_from(p.C + c * p.Ra + r, p.zstride, p.ra, p.out, p.n, e);
    else
      rescale_from(p.Cb + c * p.Rb + (r - p.split), p.zstride_b, p.ra, p.out, p.n, e);
  }
}

// ra is indexed by database slot.
__global__ void __launch_bounds__(kChunk) k_crt_rns_batched(const BatchElemHeader* hdr, const BatchCrtDesc* d,
                                                            RnsCrtArgs ra) {
  __shared__ int64_t begins[kMaxBatch + kMaxPrimes];  // one entry per problem (items + split levels)
  const int n = hdr->n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) begins[i] = d[i].elem_begin;
  __syncthreads();
  const int64_t total = hdr->total;
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < total; base += (int64_t)gridDim.x * kChunk) {
    const int b = find_problem(begins, n, base);
    const BatchCrtDesc& p = d[b];
    const int64_t nq = (p.n + 3) / 4;  // units: 4 consecutive entries of one prime slot
    const int64_t e = base + threadIdx.x - p.elem_begin;
    if (e >= (int64_t)p.nz * nq) continue;
    int z = 0;
    int64_t i = e;
    while (i >= nq) {  // nz is at most the number of primes
      i -= nq;
      ++z;
    }
    const int slot = z < p.level ? z : p.pslot;
    crt_quad(p.res + (size_t)z * ra.n * p.n, p.n, ra, slot, p.C + (size_t)z * p.n, 4 * i);
  }
}

hipError_t launch_lift_batched(const BatchElemHeader* hdr, const BatchLiftDesc* d, int64_t K, int64_t KB, int form,
                               int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_lift_batched, dim3((unsigned)grid), dim3(kChunk), 0, s, hdr, d, K, KB, form);
  return hipGetLastError();
}

hipError_t launch_rescale_batched(const BatchElemHeader* hdr, const BatchRescaleDesc* d, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_rescale_batched, dim3((unsigned)grid), dim3(kChunk), 0, s, hdr, d);
  return hipGetLastError();
}

hipError_t launch_crt_rns_batched(const BatchElemHeader* hdr, const BatchCrtDesc* d, const RnsCrtArgs& ra, int grid,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_crt_rns_batched, dim3((unsigned)grid), dim3(kChunk), 0, s, hdr, d, ra);
  return hipGetLastError();
}

}  // namespace hfe
