// The modular contraction of the CCMM (Section 2.3: the four plaintext matrix products, written
// as one product D X per prime; Section 6.3 reduces them to small-integer matrix products).
//
//   C[z][c][r] = sum_k D_z[src(r)][k] X_z[c][k]  mod prime_z
//
// for the prime slots z (the level's query primes, then p), query columns c < d3 and output
// rows r < R_out = N_DB + rows, where output rows map to database rows
// src(r) = r (A-part) for r < N_DB and N_DB + row0 + (r - N_DB) (the selected codes).
//
// Two forms, bit-identical results:
//  * plain: residues < 2^36 split into 18-bit limbs, limb products accumulated exactly in
//    64-bit integers on the vector ALU, one reduction per output;
//  * i8: centered residues split into 5 balanced int8 digits; the 25 digit-pair products run
//    on int8 MFMA (v_mfma_i32_32x32x32_i8) with the pairs of equal weight 256^(s+t) sharing
//    one int32 accumulator (9 accumulators), exact because a K-chunk of at most 32,704
//    keeps every partial sum below 2^31; recombination by Horner's rule in 64-bit integers
//    with a Barrett reduction at each step.
#include "hfe_internal.h"

namespace hfe {

__device__ __forceinline__ int64_t src_row(int64_t r, int64_t n_db, int64_t row0) {
  return r < n_db ? r : r + row0;
}

// ------------------------------------------------------------------ plain form
constexpr int kPR = 64;   // output rows per workgroup (one per lane)
constexpr int kPC = 32;   // query columns per workgroup (8 per wave)
constexpr int kPK = 16;   // K step

__global__ void __launch_bounds__(256) k_gemm_plain(GemmArgs g) {
  __shared__ uint2 sD[kPK][kPR];
  __shared__ uint2 sX[kPK][kPC];
  const int z = blockIdx.z;
  const uint64_t* __restrict__ Dt = g.Dt[z];
  const uint64_t* __restrict__ X = g.X[z];
  const int64_t r0 = (int64_t)blockIdx.x * kPR, c0 = (int64_t)blockIdx.y * kPC;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  // D loads: element e = tid + 256 i, kk = e / 64, rr = e % 64 -> rr = tx, kk = ty + 4 i
  const int64_t r_ld = r0 + tx;
  const bool r_ok = r_ld < g.R_out;
  const int64_t src = r_ok ? src_row(r_ld, g.n_db, g.row0) : 0;
  // X loads: e = tid + 256 i (i < 2), cc = e / 16, kk = e % 16
  const int kk_x = tid & 15;
  const int cc_x0 = tid >> 4, cc_x1 = (tid + 256) >> 4;
  uint64_t acc[8][3];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0;
  const uint32_t m18 = (1u << 18) - 1;
  for (int64_t k0 = 0; k0 < g.K; k0 += kPK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = ty + 4 * i;
      const int64_t k = k0 + kk;
      const uint64_t v = (r_ok && k < g.K) ? Dt[k * g.R_db + src] : 0;
      sD[kk][tx] = make_uint2((uint32_t)v & m18, (uint32_t)(v >> 18));
    }
    {
      const int64_t k = k0 + kk_x;
      const int64_t ca = c0 + cc_x0, cb = c0 + cc_x1;
      const uint64_t va = (ca < g.d3 && k < g.K) ? X[ca * g.K + k] : 0;
      const uint64_t vb = (cb < g.d3 && k < g.K) ? X[cb * g.K + k] : 0;
      sX[kk_x][cc_x0] = make_uint2((uint32_t)va & m18, (uint32_t)(va >> 18));
      sX[kk_x][cc_x1] = make_uint2((uint32_t)vb & m18, (uint32_t)(vb >> 18));
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kPK; ++kk) {
      const uint2 d = sD[kk][tx];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint2 x = sX[kk][ty * 8 + j];
        acc[j][0] += (uint64_t)d.x * x.x;
        acc[j][1] += (uint64_t)d.x * x.y + (uint64_t)d.y * x.x;
        acc[j][2] += (uint64_t)d.y * x.y;
      }
    }
    __syncthreads();
  }
  const Mod m = g.mod[z];
  const uint64_t c36 = barrett64(1ull << 36, m.q, m.mu);
  const uint64_t c36_sh = shoup_quot(c36, m.q);
  if (!r_ok) return;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t c = c0 + ty * 8 + j;
    if (c >= g.d3) continue;
    const uint64_t lo = barrett64(acc[j][0], m.q, m.mu);
    const uint64_t mid = barrett64(barrett64(acc[j][1], m.q, m.mu) << 18, m.q, m.mu);
    const uint64_t hi = mul_shoup(barrett64(acc[j][2], m.q, m.mu), c36, c36_sh, m.q);
    g.C[z][c * g.R_out + r_ld] = add_mod(add_mod(lo, mid, m.q), hi, m.q);
  }
}

hipError_t launch_gemm_plain(const GemmArgs& g, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.R_out + kPR - 1) / kPR), (unsigned)((g.d3 + kPC - 1) / kPC), (unsigned)g.nz);
  hipLaunchKernelGGL(k_gemm_plain, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ int8 MFMA form
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kIQ = 64;           // query columns per workgroup (2 waves x 32)
constexpr int kIR = 64;           // output rows per workgroup (2 waves x 32)
constexpr int kLdsRow = 80;       // bytes per LDS row: 64 digits + 16 pad (conflict-free b128 reads)
constexpr int kChunkKB = 511;     // K-blocks per exact int32 chunk: 511 * 64 * 4 * 2^14 < 2^31

// Horner recombination of the 9 anti-diagonal sums a_u (weight 256^u) into a residue:
// r <- (r * 256 + a_u + q) mod q from u = 8 down to 0.  |a_u| < 2^31 < q, so every
// intermediate is in [0, 257 q + 2^31) < 2^45.
__device__ __forceinline__ uint64_t horner9(const int32_t a[9], uint64_t q, uint64_t mu) {
  uint64_t r = 0;
#pragma unroll
  for (int u = 8; u >= 0; --u) {
    const uint64_t x = (r << 8) + (uint64_t)((int64_t)a[u] + (int64_t)q);
    r = barrett64(x, q, mu);
  }
  return r;
}

// Tile schedule: the workgroups of one launch are dealt round-robin to the 8 XCDs (each with its
// own L2).  Workgroup i runs on XCD i % 8; its tile is chosen so that one XCD receives all
// query-column tiles of a database-row tile back to back, hence the database digits of that
// tile are fetched from HBM once into that XCD's L2 and shared by its query-column tiles.
constexpr int kXcds = 8;

__global__ void __launch_bounds__(256) k_gemm_i8(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) int8_t sA[2][kDigits][kIQ][kLdsRow];  // query digits
  __shared__ __attribute__((aligned(16))) int8_t sB[2][kDigits][kIR][kLdsRow];  // database digits
  const int z = blockIdx.z;
  const int64_t n_ct = (g.d3 + kIQ - 1) / kIQ, n_rt = (g.R_out + kIR - 1) / kIR;
  const int64_t wg = blockIdx.x, xcd = wg % kXcds, j = wg / kXcds;
  const int64_t rt = (j / n_ct) * kXcds + xcd, ct = j % n_ct;
  if (rt >= n_rt) return;
  const int8_t* __restrict__ Xd = g.Xd[z];
  const int8_t* __restrict__ Dd = g.Dd[z];
  const int64_t r0 = rt * kIR, c0 = ct * kIQ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave & 1, wr = wave >> 1;
  // global -> LDS: thread loads 16 bytes (chunk tid & 3) of row (tid >> 2) of each digit plane
  const int ld_row = tid >> 2, ld_chunk = tid & 3;
  const int64_t db_row = src_row(r0 + ld_row, g.n_db, g.row0);  // < R_pad for every tile (padding)
  const int64_t q_col = c0 + ld_row;                            // < d3_pad
  const size_t planeB = (size_t)g.KB * g.R_pad * kKB, planeA = (size_t)g.KB * g.d3_pad * kKB;
  const size_t stepB = (size_t)g.R_pad * kKB, stepA = (size_t)g.d3_pad * kKB;
  const int8_t* gB = Dd + (size_t)db_row * kKB + ld_chunk * 16;
  const int8_t* gA = Xd + (size_t)q_col * kKB + ld_chunk * 16;
  const Mod m = g.mod[z];
  // 32x32 MFMA result layout: lane l, element j holds row (M = query) 8 (j / 4) + 4 (l / 32)
  // + j % 4 and column (N = database row) l % 32.
  const int64_t out_r = r0 + wr * 32 + (lane & 31);
  uint64_t* C = g.C[z];

  for (int64_t kb0 = 0; kb0 < g.KB; kb0 += kChunkKB) {
    const int64_t kb1 = kb0 + kChunkKB < g.KB ? kb0 + kChunkKB : g.KB;
    v16i acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    v4i pa[kDigits], pb[kDigits];
#pragma unroll
    for (int t = 0; t < kDigits; ++t) {
      pa[t] = *reinterpret_cast<const v4i*>(gA + t * planeA + kb0 * stepA);
      pb[t] = *reinterpret_cast<const v4i*>(gB + t * planeB + kb0 * stepB);
    }
#pragma unroll
    for (int t = 0; t < kDigits; ++t) {
      *reinterpret_cast<v4i*>(&sA[kb0 & 1][t][ld_row][ld_chunk * 16]) = pa[t];
      *reinterpret_cast<v4i*>(&sB[kb0 & 1][t][ld_row][ld_chunk * 16]) = pb[t];
    }
    __syncthreads();
    for (int64_t kb = kb0; kb < kb1; ++kb) {
      const int cur = (int)(kb & 1);
      const bool more = kb + 1 < kb1;
      if (more) {
        const size_t offA = (size_t)(kb + 1) * stepA, offB = (size_t)(kb + 1) * stepB;
#pragma unroll
        for (int t = 0; t < kDigits; ++t) {
          pa[t] = *reinterpret_cast<const v4i*>(gA + t * planeA + offA);
          pb[t] = *reinterpret_cast<const v4i*>(gB + t * planeB + offB);
        }
      }
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int koff = half * 32 + (lane >> 5) * 16;
        v4i a[kDigits];
#pragma unroll
        for (int t = 0; t < kDigits; ++t)
          a[t] = *reinterpret_cast<const v4i*>(&sA[cur][t][wq * 32 + (lane & 31)][koff]);
#pragma unroll
        for (int s = 0; s < kDigits; ++s) {
          const v4i b = *reinterpret_cast<const v4i*>(&sB[cur][s][wr * 32 + (lane & 31)][koff]);
#pragma unroll
          for (int t = 0; t < kDigits; ++t)
            acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[t], b, acc[s + t], 0, 0, 0);
        }
      }
      if (more) {
#pragma unroll
        for (int t = 0; t < kDigits; ++t) {
          *reinterpret_cast<v4i*>(&sA[cur ^ 1][t][ld_row][ld_chunk * 16]) = pa[t];
          *reinterpret_cast<v4i*>(&sB[cur ^ 1][t][ld_row][ld_chunk * 16]) = pb[t];
        }
      }
      __syncthreads();
    }
    // Recombine this K-chunk and accumulate it into the output (first chunk stores).
    if (out_r < g.R_out) {
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int64_t c = c0 + wq * 32 + 8 * (jj >> 2) + 4 * (lane >> 5) + (jj & 3);
        if (c >= g.d3) continue;
        int32_t a9[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) a9[u] = acc[u][jj];
        uint64_t v = horner9(a9, m.q, m.mu);
        uint64_t* dst = C + c * g.R_out + out_r;
        if (kb0) v = add_mod(v, *dst, m.q);
        *dst = v;
      }
    }
  }
}

hipError_t launch_gemm_i8(const GemmArgs& g, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  const int64_t n_ct = (g.d3 + kIQ - 1) / kIQ, n_rt = (g.R_out + kIR - 1) / kIR;
  const int64_t n_rt8 = (n_rt + kXcds - 1) / kXcds * kXcds;
  dim3 grid((unsigned)(n_rt8 * n_ct), 1, (unsigned)g.nz);
  hipLaunchKernelGGL(k_gemm_i8, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace hfe
