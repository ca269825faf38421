// n^2 int8 form of the modular contraction (Section 6.3: a matrix modulo n^2 written as M + n M'
// with small entries, so that its product modulo n^2 follows from three int8 products,
// M N + n (M N' + M' N)).  For a prime q of the basis, C = D X mod q is recovered from the exact
// integer sum S = sum_k d_k x_k of centered residues: S mod n_j^2 for a few prime bases
// 211 <= n_j <= 251 (three int8 products each, two int32 accumulators), then the CRT of those
// residues to S (the product of the n_j^2 is at least 4 |S|), then S mod q.
#include "hfe_device.h"

namespace hfe {

// ------------------------------------------------------------------ database split
// Thread (row r, K-block kb): the 64 centered residues of D[k][r] -> per base one 64-byte row of M
// (plane 2j) and one of M' (plane 2j + 1).
__global__ void __launch_bounds__(256) k_split_db_p2(const uint64_t* Dt, int64_t K, int64_t R, int64_t KB,
                                                     int64_t R_pad, uint64_t q, int n_bases, int8_t* planes) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kb = blockIdx.y;
  if (r >= R_pad) return;
  int64_t x[kKB];
#pragma unroll
  for (int kk = 0; kk < kKB; ++kk) {
    const int64_t k = kb * kKB + kk;
    x[kk] = (r < R && k < K) ? centered(Dt[k * R + r], q) : 0;
  }
  for (int j = 0; j < n_bases; ++j) {
    uint4* d0 = reinterpret_cast<uint4*>(planes + (((int64_t)(2 * j) * KB + kb) * R_pad + r) * kKB);
    uint4* d1 = reinterpret_cast<uint4*>(planes + (((int64_t)(2 * j + 1) * KB + kb) * R_pad + r) * kKB);
#pragma unroll
    for (int i = 0; i < kKB / 16; ++i) {  // 16 bytes of each plane at a time
      uint32_t w0[4], w1[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint32_t v0 = 0, v1 = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          int32_t M, Mp;
          p2_digits(x[16 * i + 4 * t + b], j, M, Mp);
          v0 |= ((uint32_t)M & 255u) << (8 * b);
          v1 |= ((uint32_t)Mp & 255u) << (8 * b);
        }
        w0[t] = v0;
        w1[t] = v1;
      }
      d0[i] = make_uint4(w0[0], w0[1], w0[2], w0[3]);
      d1[i] = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    }
  }
}

hipError_t launch_split_db_p2(const uint64_t* Dt_prime, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                              uint64_t q, int n_bases, int8_t* planes_prime, hipStream_t s) {
  if (n_bases < 1 || n_bases > kP2MaxBases) return hipErrorInvalidValue;
  dim3 grid((unsigned)((R_pad + 255) / 256), (unsigned)KB);
  hipLaunchKernelGGL(k_split_db_p2, grid, dim3(256), 0, s, Dt_prime, K, R, KB, R_pad, q, n_bases, planes_prime);
  return hipGetLastError();
}

// ------------------------------------------------------------------ query lift
// Element (c, k): the lift of the query residues (as for the digit form), then for every prime of
// the level and p the digits M, M' of the centered value for each base: Xq[z][2j + t][kb][c][kk],
// zero in the padding.
__global__ void __launch_bounds__(256) k_lift_p2(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                                 int64_t d3_pad, LiftArgs la, int n_bases, int8_t* Xq) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= KB * kKB) return;
  lift_lane(XT, d3, K, KB, d3_pad, la, -n_bases, nullptr, Xq, blockIdx.y, k);
}

hipError_t launch_lift_p2(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                          const LiftArgs& la, int n_bases, int8_t* Xq, hipStream_t s) {
  if (n_bases < 1 || n_bases > kP2MaxBases) return hipErrorInvalidValue;
  dim3 grid((unsigned)((KB * kKB + 255) / 256), (unsigned)d3_pad);
  hipLaunchKernelGGL(k_lift_p2, grid, dim3(256), 0, s, XT, d3, K, KB, d3_pad, la, n_bases, Xq);
  return hipGetLastError();
}

// ------------------------------------------------------------------ contraction per base
// Workgroup tile: TR database rows x TQ query columns of one (prime, base), TQ x TR = 128 x 256 or
// 256 x 128, 8 waves (two per SIMD), each owning 64 query columns x 64 rows as 2 x 2 blocks of
// 32 x 32 with two int32 accumulators: G0 += M N and G1 += M N' + M' N (v_mfma_i32_32x32x32_i8),
// three MFMAs per block and K-chunk.  An LDS stage holds one 64-byte K-block of both query planes
// (2 x TQ rows) and both database planes (2 x TR rows), 48 KiB, fed by direct global-to-LDS loads
// with the digit form's row swizzle; three stages (144 KiB, one workgroup per CU).  Per K-block the
// workgroup loads 48 KiB for 96 MFMAs, the same bytes per MFMA as the RNS tile of 256 x 256.  The
// host takes the 128-column tile when it pads the query columns less (small problems of a batch).
// Exactness: |M|, |M'|, |N|, |N'| <= 125, so |G1| <= 2 K 125^2 < 2^31 for K <= 2^16 (checked by the
// host).
template <int TQ_>
struct P2Cfg {
  static_assert(TQ_ == 128 || TQ_ == 256, "query tile of 128 or 256 columns");
  static constexpr int TQ = TQ_, TR = 128 * 256 / TQ_;
  static constexpr int WQB = 2, WRB = 2;  // 32 x 32 blocks per wave
  static constexpr int NQ = TQ / (32 * WQB), NR = TR / (32 * WRB), NW = NQ * NR;
  static constexpr int STAGES = 3;
  static constexpr int PA = 2 * TQ * kKB, PB = 2 * TR * kKB, STAGE = PA + PB;
  static constexpr int LA = 2 * TQ / 16 / NW, LB = 2 * TR / 16 / NW;  // loads per wave per K-block
  static constexpr int VM = (LA + LB) * (STAGES - 2);
  static constexpr int LDS = STAGES * STAGE;
  static_assert(NW == 8 && VM == 6, "the K-block wait below is written for 6 loads in flight");
  static_assert(TQ % (16 * NW) == 0 && TR % (16 * NW) == 0, "whole loads per wave and plane");
};

// One output tile (rows r0.., query columns c0..) of one (prime, base j) product: X and D are the
// base's plane M of the query and of the database (M' follows one plane later), res its residue
// plane [d3][R_out].
struct P2Tile {
  const int8_t* X;
  const int8_t* D;
  uint16_t* res;
  int j;
  int32_t bn, bm;        // the base n and n^2 of this product
  double brn, brm;       // RN(1 / n), RN(1 / n^2)
  int64_t KB, R_pad, d3_pad, n_db, row0, R_out, d3, r0, c0;
};

template <int TQ>
__device__ __forceinline__ void p2_tile(const P2Tile& g, int8_t* lds) {
  using C = P2Cfg<TQ>;
  const int64_t r0 = g.r0, c0 = g.c0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wq = wave % C::NQ, wr = wave / C::NQ;
  const int8_t* X = g.X;
  const int8_t* D = g.D;
  const size_t planeA = (size_t)g.KB * g.d3_pad * kKB, planeB = (size_t)g.KB * g.R_pad * kKB;
  const size_t stepA = (size_t)g.d3_pad * kKB, stepB = (size_t)g.R_pad * kKB;
  // Load i of a wave fills stage row u = 16 (wave + NW i) + lane / 4 of the stacked planes (u / T
  // is the plane, u % T the tile row), chunk (lane % 4) ^ ((u >> 2) & 3).
  const int ld_row = 16 * wave + (lane >> 2);
  const int ld_chunk = ((lane & 3) ^ ((ld_row >> 2) & 3)) * 16;
  const int8_t* gA[C::LA];
  const int8_t* gB[C::LB];
#pragma unroll
  for (int i = 0; i < C::LA; ++i) {
    const int u = ld_row + 16 * C::NW * i;
    gA[i] = X + (u / C::TQ) * planeA + (size_t)(c0 + u % C::TQ) * kKB + ld_chunk;
  }
#pragma unroll
  for (int i = 0; i < C::LB; ++i) {
    const int u = ld_row + 16 * C::NW * i;
    gB[i] = D + (u / C::TR) * planeB + (size_t)src_row(r0 + u % C::TR, g.n_db, g.row0) * kKB + ld_chunk;
  }
  const uint32_t lds0 = (uint32_t)(uintptr_t)lds + wave * 16 * kKB;
  auto issue = [&](int stage, int64_t kb) {
    const uint32_t base = lds0 + stage * C::STAGE;
#pragma unroll
    for (int i = 0; i < C::LA; ++i) dma16(gA[i] + kb * stepA, base + 16 * C::NW * i * kKB);
#pragma unroll
    for (int i = 0; i < C::LB; ++i) dma16(gB[i] + kb * stepB, base + C::PA + 16 * C::NW * i * kKB);
  };
  const int sw = ((lane & 31) >> 2) & 3, cl = lane >> 5;
  const int offA = (wq * 32 * C::WQB + (lane & 31)) * kKB;            // plane M rows; M' at + TQ rows
  const int offB = C::PA + (wr * 32 * C::WRB + (lane & 31)) * kKB;    // plane N rows; N' at + TR rows
  v16i acc0[C::WQB][C::WRB], acc1[C::WQB][C::WRB];
#pragma unroll
  for (int a = 0; a < C::WQB; ++a)
#pragma unroll
    for (int b = 0; b < C::WRB; ++b) {
      acc0[a][b] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      acc1[a][b] = acc0[a][b];
    }
  const int64_t KB = g.KB;
  auto clamp = [&](int64_t i) { return i < KB ? i : KB - 1; };
  // fragments of one half (32 bytes of K) of the K-block in stage st: [0] the M / N plane, [1] M' / N'
  struct Frags {
    v4i a[2][C::WQB], b[2][C::WRB];
  };
  auto read_half = [&](int st, int h, Frags& f) {
    const int8_t* S = lds + st * C::STAGE;
    const int chunk = ((cl + 2 * h) ^ sw) << 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int a = 0; a < C::WQB; ++a)
        f.a[t][a] = *reinterpret_cast<const v4i*>(S + offA + (t * C::TQ + a * 32) * kKB + chunk);
#pragma unroll
      for (int b = 0; b < C::WRB; ++b)
        f.b[t][b] = *reinterpret_cast<const v4i*>(S + offB + (t * C::TR + b * 32) * kKB + chunk);
    }
  };
  // G0 += M N and the first term of G1 for every block, then the second term of G1, so that the two
  // products into one G1 accumulator are not back to back
  auto mma = [&](const Frags& f) {
#pragma unroll
    for (int a = 0; a < C::WQB; ++a)
#pragma unroll
      for (int b = 0; b < C::WRB; ++b) {
        acc0[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[0][a], f.b[0][b], acc0[a][b], 0, 0, 0);
        acc1[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[0][a], f.b[1][b], acc1[a][b], 0, 0, 0);
      }
#pragma unroll
    for (int a = 0; a < C::WQB; ++a)
#pragma unroll
      for (int b = 0; b < C::WRB; ++b)
        acc1[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[1][a], f.b[0][b], acc1[a][b], 0, 0, 0);
  };
  // software pipeline as in the RNS tile: half 1 is read while half 0 multiplies, half 0 of the next
  // K-block while half 1 multiplies; the barrier between the halves frees the oldest stage
#pragma unroll
  for (int st = 0; st < C::STAGES - 1; ++st) issue(st, clamp(st));
  asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  issue(C::STAGES - 1, clamp(C::STAGES - 1));
  Frags f0, f1;
  read_half(0, 0, f0);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt untouched
  int cur = 0;
  for (int64_t i = 0; i < KB; ++i) {
    read_half(cur, 1, f1);
    __builtin_amdgcn_sched_barrier(0);
    mma(f0);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    issue(cur, clamp(i + C::STAGES));
    cur = cur + 1 == C::STAGES ? 0 : cur + 1;
    read_half(cur, 0, f0);  // block i + 1 (a landed duplicate of the last block at the end)
    __builtin_amdgcn_sched_barrier(0);
    mma(f1);
    __builtin_amdgcn_sched_barrier(0);
  }
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  // epilogue: S mod n^2 = (G0 mod n^2 + n (G1 mod n)) mod n^2 -> res[z][j][c][r]; 32 x 32 result
  // layout as in the digit form (lane l, element e: query column 8 (e / 4) + 4 (l / 32) + e % 4,
  // row l % 32)
  const int32_t n = g.bn, m = g.bm;
  const double rn = g.brn, rm = g.brm;
  uint16_t* res = g.res;
#pragma unroll
  for (int b = 0; b < C::WRB; ++b) {
    const int64_t r = r0 + wr * 32 * C::WRB + b * 32 + (lane & 31);
    if (r >= g.R_out) continue;
#pragma unroll
    for (int a = 0; a < C::WQB; ++a)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t c = c0 + wq * 32 * C::WQB + a * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (c >= g.d3) continue;
        res[c * g.R_out + r] = (uint16_t)p2_acc_mod(acc0[a][b][e], acc1[a][b][e], n, m, rn, rm);
      }
  }
}

template <int TQ>
__global__ void __launch_bounds__(64 * P2Cfg<TQ>::NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_p2(P2GemmArgs g) {
  using C = P2Cfg<TQ>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C::LDS];
  const int j = blockIdx.y, z = blockIdx.z;
  const int64_t n_ct = (g.d3 + C::TQ - 1) / C::TQ, n_rt = (g.R_out + C::TR - 1) / C::TR;
  const int64_t l = blockIdx.x, xcd = l % kXcds, jj = l / kXcds;
  const int64_t rt = (jj / n_ct) * kXcds + xcd, ct = jj % n_ct;
  if (rt >= n_rt) return;
  P2Tile t{g.Xq[z] + (size_t)(2 * j) * g.KB * g.d3_pad * kKB, g.Dq[z] + (size_t)(2 * j) * g.KB * g.R_pad * kKB,
           g.res + ((size_t)z * g.n_bases + j) * g.d3 * g.R_out, j, g.n[j], g.m[j], g.rn[j], g.rm[j], g.KB, g.R_pad,
           g.d3_pad, g.n_db, g.row0, g.R_out, g.d3, rt * C::TR, ct * C::TQ};
  p2_tile<TQ>(t, lds);
}

// Persistent batched form: problem b's tiles are ordered (z, base, XCD-ordered tile), starting at its
// tile_begin; workgroups claim tiles in order from one counter per XCD (tile t = 8 i + xcd), as the
// digit form's batched kernel.  The 256-column launch serves problems [0, n_wide) (tiles
// [0, tiles_wide), counters next), the 128-column launch the others (counters next_narrow).
template <int TQ>
__global__ void __launch_bounds__(64 * P2Cfg<TQ>::NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_p2_batched(P2BatchArgs a) {
  using C = P2Cfg<TQ>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C::LDS];
  constexpr bool narrow = TQ == 128;
  const int p_lo = narrow ? a.hdr->n_wide : 0, p_hi = narrow ? a.hdr->n : a.hdr->n_wide;
  const int64_t t_lo = narrow ? a.hdr->tiles_wide : 0, t_hi = narrow ? a.hdr->total_tiles : a.hdr->tiles_wide;
  uint32_t* next = narrow ? a.next_narrow : a.next;
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = (t_hi - t_lo) / kXcds;
  for (;;) {
    __syncthreads();  // the previous tile is done with LDS
    if (threadIdx.x == 0) *reinterpret_cast<uint32_t*>(lds) = atomicAdd(next + xcd, 1u);
    __syncthreads();
    const int64_t jc = (uint32_t)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const uint32_t*>(lds));
    __syncthreads();  // every thread has read the claim before the tile overwrites LDS
    if (jc >= per_xcd) break;
    const int64_t t = t_lo + jc * kXcds + xcd;
    int lo = p_lo, hi = p_hi - 1;  // last problem of this launch whose first tile is <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.desc[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const BatchDesc& d = a.desc[lo];
    const int64_t n_ct = (d.d3 + C::TQ - 1) / C::TQ, n_rt = (d.R_out + C::TR - 1) / C::TR;
    const int64_t per_base = (n_rt + kXcds - 1) / kXcds * kXcds * n_ct;
    const int64_t local = t - d.tile_begin;
    const int zj = (int)(local / per_base);
    const int z = zj / a.n_bases, j = zj % a.n_bases;
    const int64_t l = local % per_base, lj = l / kXcds;
    const int64_t rt = (lj / n_ct) * kXcds + l % kXcds, ct = lj % n_ct;
    if (rt >= n_rt) continue;
    P2Tile tl{d.Xd + (size_t)(z * a.n_bases + j) * 2 * a.KB * d.d3_pad * kKB,
              a.Dq + (size_t)(d.slot[z] * a.n_bases + j) * 2 * a.KB * a.R_pad * kKB,
              reinterpret_cast<uint16_t*>(d.res) + ((size_t)z * a.n_bases + j) * d.d3 * d.R_out, j, kP2C.n[j],
              kP2C.m[j], kP2C.rcp_n[j], kP2C.rcp_m[j], a.KB, a.R_pad, d.d3_pad, d.n_db, d.row0, d.R_out, d.d3,
              rt * C::TR, ct * C::TQ};
    p2_tile<TQ>(tl, lds);
  }
}

static int64_t p2_rows_of(int tq) { return 128 * 256 / tq; }

int64_t p2_batched_tiles(int64_t d3, int64_t R_out, int nz, int n_bases, int tq) {
  const int64_t tr = p2_rows_of(tq);
  const int64_t n_ct = (d3 + tq - 1) / tq, n_rt = (R_out + tr - 1) / tr;
  return (n_rt + kXcds - 1) / kXcds * kXcds * n_ct * nz * n_bases;
}

// Query tile of the n^2 contraction for a set of problems: the width with less padded work (rows
// padded to the tile's TR, columns to its TQ); ties go to 256.
int p2_tile_q(const int64_t* d3, const int64_t* R_out, const int* nz, int n) {
  double w128 = 0, w256 = 0;
  for (int i = 0; i < n; ++i) {
    w128 += (double)((R_out[i] + 255) / 256 * 256) * ((d3[i] + 127) / 128 * 128) * nz[i];
    w256 += (double)((R_out[i] + 127) / 128 * 128) * ((d3[i] + 255) / 256 * 256) * nz[i];
  }
  return w128 < w256 ? 128 : 256;
}

hipError_t launch_gemm_p2_batched(const P2BatchArgs& a, int grid, int tq, hipStream_t s) {
  if (tq == 128)
    hipLaunchKernelGGL(k_gemm_p2_batched<128>, dim3((unsigned)grid), dim3(64 * P2Cfg<128>::NW), 0, s, a);
  else if (tq == 256)
    hipLaunchKernelGGL(k_gemm_p2_batched<256>, dim3((unsigned)grid), dim3(64 * P2Cfg<256>::NW), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gemm_p2(const P2GemmArgs& g, int tq, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  if ((tq != 128 && tq != 256) || g.d3_pad % tq != 0 || g.n_bases < 1 || g.n_bases > kP2ArgBases)
    return hipErrorInvalidValue;
  const int64_t tr = p2_rows_of(tq);
  const int64_t n_ct = (g.d3 + tq - 1) / tq, n_rt = (g.R_out + tr - 1) / tr;
  const int64_t n_rt8 = (n_rt + kXcds - 1) / kXcds * kXcds;
  dim3 grid((unsigned)(n_rt8 * n_ct), (unsigned)g.n_bases, (unsigned)g.nz);
  if (tq == 128)
    hipLaunchKernelGGL(k_gemm_p2<128>, grid, dim3(64 * P2Cfg<128>::NW), 0, s, g);
  else
    hipLaunchKernelGGL(k_gemm_p2<256>, grid, dim3(64 * P2Cfg<256>::NW), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ CRT back to the prime
// Entry e of prime slot z: residues s_j = S mod m_j (m_j = n_j^2).  As in the RNS form's CRT, with
// y_j = s_j (M/m_j)^-1 mod m_j: S = sum_j y_j (M/m_j) - a M with a = round(sum_j y_j / m_j), which
// single precision decides because M >= 4 max |S| (the fraction lies at least 1/4 from 1/2 and the
// float sum of at most 8 terms is off by less than 2^-20); then
// C = sum_j y_j ((M/m_j) mod q) - a (M mod q) mod q, the sum below 8 * 2^16 * 2^36.
// Thread: 2 consecutive entries of one prime slot (blockIdx.y), residues read as one 4-byte word.
// Entries e0, e0 + 1 (those below n) of one prime slot: r = that slot's first residue plane
// ([n_bases][n] uint16); ra indexed by `slot`.  v[b] = entry e0 + b (v[1] is 0 past the end).
__device__ __forceinline__ void crt_pair_vals(const uint16_t* r, int64_t n, const P2CrtArgs& ra, int slot,
                                              int64_t e0, uint64_t v[2]) {
  const int cnt = e0 + 1 < n ? 2 : 1;
  float frac[2] = {0.f, 0.f};
  uint64_t acc[2] = {0, 0};
  for (int j = 0; j < ra.n; ++j) {
    uint32_t s2[2];
    if (cnt == 2 && (n & 1) == 0) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(r + (size_t)j * n + e0);
      s2[0] = w & 0xFFFFu;
      s2[1] = w >> 16;
    } else {
      s2[0] = r[(size_t)j * n + e0];
      s2[1] = cnt == 2 ? r[(size_t)j * n + e0 + 1] : 0u;
    }
    const int64_t m = ra.m[j];
    const double rcp = 1.0 / (double)m;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint32_t y = (uint32_t)mod_f64((int64_t)s2[b] * ra.inv[j], m, rcp);
      frac[b] = crt_frac_add(frac[b], y, ra.rcp[j]);
      acc[b] += (uint64_t)y * ra.Mj_mod_q[slot][j];
    }
  }
  const Mod md = ra.mod[slot];
  v[1] = 0;
  for (int b = 0; b < cnt; ++b) v[b] = crt_finish(acc[b], crt_round(frac[b]), ra.M_mod_q[slot], md);
}

// The same, stored: out = the slot's n results.
__device__ __forceinline__ void crt_pair(const uint16_t* r, int64_t n, const P2CrtArgs& ra, int slot, uint64_t* out,
                                         int64_t e0) {
  uint64_t v[2];
  crt_pair_vals(r, n, ra, slot, e0, v);
  out[e0] = v[0];
  if (e0 + 1 < n) out[e0 + 1] = v[1];
}

// CRT and rescale by p in one pass (single calls), as k_crt_rescale_rns: the contraction output C
// is never written.  Thread: 2 consecutive entries.
__global__ void __launch_bounds__(256) k_crt_rescale_p2(const uint16_t* res, int64_t n, P2CrtArgs ra, RescaleArgs rs,
                                                        uint64_t* out) {
  const int level = rs.level;
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (e0 >= n) return;
  const bool two = e0 + 1 < n;
  uint64_t v[2];
  crt_pair_vals(res + (size_t)level * ra.n * n, n, ra, level, e0, v);
  const int64_t cp0 = centered(v[0], rs.p), cp1 = centered(v[1], rs.p);
  for (int i = 0; i < level; ++i) {
    crt_pair_vals(res + (size_t)i * ra.n * n, n, ra, i, e0, v);
    out[(size_t)i * n + e0] = rescale_value(v[0], cp0, rs, i);
    if (two) out[(size_t)i * n + e0 + 1] = rescale_value(v[1], cp1, rs, i);
  }
}

hipError_t launch_crt_rescale_p2(const uint16_t* res, int64_t n, const P2CrtArgs& ra, const RescaleArgs& rs,
                                 uint64_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 2 * 256 - 1) / (2 * 256);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_crt_rescale_p2, dim3((unsigned)blocks), dim3(256), 0, s, res, n, ra, rs, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_crt_p2(const uint16_t* res, int64_t n, P2CrtArgs ra, uint64_t* C) {
  const int z = blockIdx.y;
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (e0 >= n) return;
  crt_pair(res + (size_t)z * ra.n * n, n, ra, z, C + (size_t)z * n, e0);
}

// Batched: every problem's residues (BatchCrtDesc, res pointing at uint16 residues), in units of 2
// entries of one prime slot; each problem's units start at a multiple of 256.  ra indexed by
// database slot.
__global__ void __launch_bounds__(256) k_crt_p2_batched(const BatchElemHeader* hdr, const BatchCrtDesc* d,
                                                        P2CrtArgs ra) {
  __shared__ int64_t begins[kMaxBatch + kMaxPrimes];  // one entry per problem (items + split levels)
  const int n = hdr->n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) begins[i] = d[i].elem_begin;
  __syncthreads();
  const int64_t total = hdr->total;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < total; base += (int64_t)gridDim.x * 256) {
    int lo = 0, hi = n - 1;  // last problem whose first unit is <= base (uniform over the block)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (begins[mid] <= base) lo = mid; else hi = mid - 1;
    }
    const BatchCrtDesc& p = d[__builtin_amdgcn_readfirstlane(lo)];
    const int64_t nq = (p.n + 1) / 2;
    const int64_t e = base + threadIdx.x - p.elem_begin;
    if (e >= (int64_t)p.nz * nq) continue;
    const int z = (int)(e / nq);
    const int64_t i = e - z * nq;
    const int slot = z < p.level ? z : p.pslot;
    crt_pair(reinterpret_cast<const uint16_t*>(p.res) + (size_t)z * ra.n * p.n, p.n, ra, slot, p.C + (size_t)z * p.n,
             2 * i);
  }
}

hipError_t launch_crt_p2_batched(const BatchElemHeader* hdr, const BatchCrtDesc* d, const P2CrtArgs& ra, int grid,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_crt_p2_batched, dim3((unsigned)grid), dim3(256), 0, s, hdr, d, ra);
  return hipGetLastError();
}

hipError_t launch_crt_p2(const uint16_t* res, int nz, int64_t n, const P2CrtArgs& ra, uint64_t* C, hipStream_t s) {
  if (nz <= 0 || n <= 0) return hipSuccess;
  const int64_t blocks = (n + 2 * 256 - 1) / (2 * 256);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_crt_p2, dim3((unsigned)blocks, (unsigned)nz), dim3(256), 0, s, res, n, ra, C);
  return hipGetLastError();
}

}  // namespace hfe
