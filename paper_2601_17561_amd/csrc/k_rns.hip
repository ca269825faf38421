// Small-modulus (RNS) int8 form of the modular contraction (Section 6.3: matrix products modulo a
// large modulus reduced to int8 products through RNS over small moduli).  For a prime q of the
// basis, C = D X mod q is recovered from the exact integer sum S = sum_k d_k x_k of centered
// residues: S mod m_j for n small pairwise coprime moduli m_j <= 256 (one int8 product each,
// int32 accumulation), then the CRT of those residues to S (the moduli's product exceeds 2 |S|),
// then S mod q.  One int8 product per modulus instead of 25 digit-pair products per prime.
#include "hfe_device.h"

namespace hfe {

// ------------------------------------------------------------------ database split
// Thread (row r, K-block kb): the 64 centered residues of D[k][r] -> one 64-byte row per modulus.
__global__ void __launch_bounds__(256) k_split_db_rns(const uint64_t* Dt, int64_t K, int64_t R, int64_t KB,
                                                      int64_t R_pad, uint64_t q, int n_mod, int8_t* dig) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kb = blockIdx.y;
  if (r >= R_pad) return;
  int64_t x[kKB];
#pragma unroll
  for (int kk = 0; kk < kKB; ++kk) {
    const int64_t k = kb * kKB + kk;
    x[kk] = (r < R && k < K) ? centered(Dt[k * R + r], q) : 0;
  }
  for (int j = 0; j < n_mod; ++j) {
    uint32_t w[kKB / 4];
#pragma unroll
    for (int i = 0; i < kKB / 4; ++i) {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) v |= ((uint32_t)(balanced_mod(x[4 * i + b], j) & 255)) << (8 * b);
      w[i] = v;
    }
    uint4* dst = reinterpret_cast<uint4*>(dig + (((int64_t)j * KB + kb) * R_pad + r) * kKB);
#pragma unroll
    for (int i = 0; i < kKB / 16; ++i) dst[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
  }
}

hipError_t launch_split_db_rns(const uint64_t* Dt_prime, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                               uint64_t q, int n_mod, int8_t* dig_prime, hipStream_t s) {
  dim3 grid((unsigned)((R_pad + 255) / 256), (unsigned)KB);
  hipLaunchKernelGGL(k_split_db_rns, grid, dim3(256), 0, s, Dt_prime, K, R, KB, R_pad, q, n_mod, dig_prime);
  return hipGetLastError();
}

// ------------------------------------------------------------------ query lift
// Element (c, k): the lift of the query residues (as for the digit form), then for every prime of
// the level and p the balanced residues of the centered value modulo each small modulus:
// Xr[z][j][kb][c][kk], zero in the padding.
__global__ void __launch_bounds__(256) k_lift_rns(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                                  int64_t d3_pad, LiftArgs la, int n_mod, int8_t* Xr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= KB * kKB) return;
  lift_lane(XT, d3, K, KB, d3_pad, la, n_mod, nullptr, Xr, blockIdx.y, k);
}

hipError_t launch_lift_rns(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                           const LiftArgs& la, int n_mod, int8_t* Xr, hipStream_t s) {
  dim3 grid((unsigned)((KB * kKB + 255) / 256), (unsigned)d3_pad);
  hipLaunchKernelGGL(k_lift_rns, grid, dim3(256), 0, s, XT, d3, K, KB, d3_pad, la, n_mod, Xr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ contraction per modulus
// Workgroup tile: 256 database rows x TQ query columns of one (prime, modulus).  Each wave owns 64
// query columns x 128 rows as 2 x 4 blocks of 32 x 32 with one int32 accumulator each
// (v_mfma_i32_32x32x32_i8), so each fragment read from LDS feeds 2 or 4 MFMAs.  One 64-byte K-block
// of both operands per LDS stage, fed by direct global-to-LDS loads (same row swizzle as the digit
// form's DMA tiles).
//   TQ = 256: 4 x 2 waves (two per SIMD), four stages of 32 KiB, one workgroup per CU; up to three
//     K-blocks are in flight while one is multiplied (three stages measured 6% slower, five no faster).
//   TQ = 128: 2 x 2 waves, three stages of 24 KiB, two workgroups per CU.  About 9% slower per
//     column than TQ = 256, but it pads query columns to 128 instead of 256; the host picks the
//     width per call or batch by padded work.
// Exactness: |S| over the K-range <= K * 128 * 128 < 2^31 for K < 2^17 (checked by the host).
template <int TQ>
struct RnsCfg {
  static_assert(TQ == 128 || TQ == 256, "query tile of 128 or 256 columns");
  static constexpr int WQB = 2, WRB = 4, WPE = 2;  // 32 x 32 blocks per wave; waves per SIMD
  static constexpr int TR = kRnsTileR;
  static constexpr int NQ = TQ / (32 * WQB), NR = TR / (32 * WRB), NW = NQ * NR;
  static constexpr int STAGES = TQ == 256 ? 4 : 3;
  static constexpr int PA = TQ * kKB, PB = TR * kKB, STAGE = PA + PB;
  static constexpr int LA = TQ / 16 / NW, LB = TR / 16 / NW;  // loads per wave per K-block
  static constexpr int VM = (LA + LB) * (STAGES - 2);         // loads a wave may leave in flight at a wait
  static constexpr int LDS = STAGES * STAGE;
  static_assert(TQ % (16 * NW) == 0 && TR % (16 * NW) == 0, "whole loads per wave");
  static_assert(STAGES >= 3, "the K-block wait leaves STAGES - 2 blocks in flight");
};

// One output tile (rows r0.., query columns c0..) of one (prime, modulus) product: X and D are that
// modulus' query and database planes, res its residue plane [d3][R_out].
struct RnsTile {
  const int8_t* X;
  const int8_t* D;
  uint8_t* res;
  int32_t m;
  uint32_t magic;
  int64_t KB, R_pad, d3_pad, n_db, row0, R_out, d3, r0, c0;
};

// this wave's loads of the oldest outstanding K-block have landed (the younger ones may still fly)
// and its LDS reads are done; then the same for every wave
template <int VM>
__device__ __forceinline__ void rns_wait_block() {
  static_assert(VM == 4 || VM == 6 || VM == 8 || VM == 12, "no K-block wait for this tile shape");
  if constexpr (VM == 4)
    asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else if constexpr (VM == 6)
    asm volatile("s_waitcnt vmcnt(6) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else if constexpr (VM == 8)
    asm volatile("s_waitcnt vmcnt(8) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else
    asm volatile("s_waitcnt vmcnt(12) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int TQ>
__device__ __forceinline__ void rns_tile(const RnsTile& g, int8_t* lds) {
  using C = RnsCfg<TQ>;
  const int64_t r0 = g.r0, c0 = g.c0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wq = wave % C::NQ, wr = wave / C::NQ;
  const int8_t* X = g.X;
  const int8_t* D = g.D;
  const size_t stepA = (size_t)g.d3_pad * kKB, stepB = (size_t)g.R_pad * kKB;
  // load i of a wave fills tile rows 16 (wave + NW i) .. + 15 (lane l: row + l / 4, stored chunk
  // l % 4 holding logical chunk (l % 4) ^ ((row >> 2) & 3))
  const int ld_row = 16 * wave + (lane >> 2);
  const int ld_chunk = ((lane & 3) ^ ((ld_row >> 2) & 3)) * 16;
  const int8_t* gA[C::LA];
  const int8_t* gB[C::LB];
#pragma unroll
  for (int i = 0; i < C::LA; ++i) gA[i] = X + (size_t)(c0 + ld_row + 16 * C::NW * i) * kKB + ld_chunk;
#pragma unroll
  for (int i = 0; i < C::LB; ++i)
    gB[i] = D + (size_t)src_row(r0 + ld_row + 16 * C::NW * i, g.n_db, g.row0) * kKB + ld_chunk;
  const uint32_t lds0 = (uint32_t)(uintptr_t)lds + wave * 16 * kKB;
  auto issue = [&](int stage, int64_t kb) {
    const uint32_t base = lds0 + stage * C::STAGE;
#pragma unroll
    for (int i = 0; i < C::LA; ++i) dma16(gA[i] + kb * stepA, base + 16 * C::NW * i * kKB);
#pragma unroll
    for (int i = 0; i < C::LB; ++i) dma16(gB[i] + kb * stepB, base + C::PA + 16 * C::NW * i * kKB);
  };
  const int sw = ((lane & 31) >> 2) & 3, cl = lane >> 5;
  const int offA = (wq * 32 * C::WQB + (lane & 31)) * kKB;
  const int offB = C::PA + (wr * 32 * C::WRB + (lane & 31)) * kKB;
  v16i acc[C::WQB][C::WRB];
#pragma unroll
  for (int a = 0; a < C::WQB; ++a)
#pragma unroll
    for (int b = 0; b < C::WRB; ++b) acc[a][b] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t KB = g.KB;
  auto clamp = [&](int64_t i) { return i < KB ? i : KB - 1; };
  // fragments of one half (32 bytes of K) of the K-block in stage st
  auto read_half = [&](int st, int h, v4i (&fa)[C::WQB], v4i (&fb)[C::WRB]) {
    const int8_t* S = lds + st * C::STAGE;
    const int chunk = ((cl + 2 * h) ^ sw) << 4;
#pragma unroll
    for (int a = 0; a < C::WQB; ++a) fa[a] = *reinterpret_cast<const v4i*>(S + offA + a * 32 * kKB + chunk);
#pragma unroll
    for (int b = 0; b < C::WRB; ++b) fb[b] = *reinterpret_cast<const v4i*>(S + offB + b * 32 * kKB + chunk);
  };
  auto mma = [&](const v4i (&fa)[C::WQB], const v4i (&fb)[C::WRB]) {
#pragma unroll
    for (int a = 0; a < C::WQB; ++a)
#pragma unroll
      for (int b = 0; b < C::WRB; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
  };
  // Software pipeline: the fragments of half 0 of block i are in registers when iteration i
  // starts; half 1 is read while half 0 multiplies, and half 0 of block i + 1 while half 1
  // multiplies, so LDS latency hides behind the MFMAs.  The barrier sits between the halves:
  // after it block i + 1 is in LDS and no wave reads block i's stage any more, which then
  // receives block i + STAGES.
#pragma unroll
  for (int st = 0; st < C::STAGES - 1; ++st) issue(st, clamp(st));
  rns_wait_block<C::VM>();
  issue(C::STAGES - 1, clamp(C::STAGES - 1));
  v4i f0a[C::WQB], f0b[C::WRB], f1a[C::WQB], f1b[C::WRB];
  read_half(0, 0, f0a, f0b);
  // settle every outstanding LDS and scalar load here, so that the compiler's wait analysis
  // enters the loop with LDS reads only and waits for the older half alone inside it
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt untouched
  int cur = 0;
  for (int64_t i = 0; i < KB; ++i) {
    read_half(cur, 1, f1a, f1b);
    __builtin_amdgcn_sched_barrier(0);
    mma(f0a, f0b);
    __builtin_amdgcn_sched_barrier(0);
    rns_wait_block<C::VM>();
    issue(cur, clamp(i + C::STAGES));
    cur = cur + 1 == C::STAGES ? 0 : cur + 1;
    read_half(cur, 0, f0a, f0b);  // block i + 1 (a landed duplicate of the last block at the end)
    __builtin_amdgcn_sched_barrier(0);
    mma(f1a, f1b);
    __builtin_amdgcn_sched_barrier(0);
  }
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  // epilogue: S mod m_j in [0, m_j) -> res[z][j][c][r]; 32 x 32 result layout as in the digit
  // form (lane l, element e: query column 8 (e / 4) + 4 (l / 32) + e % 4, row l % 32)
  const uint32_t m = (uint32_t)g.m;
  const uint32_t magic = g.magic;
  const RnsAccConsts ac = rns_acc_consts(m, magic);  // |acc| < 2^31 -> acc mod m (hfe_exact.h)
  uint8_t* res = g.res;
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
        res[c * g.R_out + r] = (uint8_t)rns_acc_mod(acc[a][b][e], m, magic, ac);
      }
  }
}

template <int TQ>
__global__ void __launch_bounds__(64 * RnsCfg<TQ>::NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_rns(RnsGemmArgs g) {
  using C = RnsCfg<TQ>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C::LDS];
  const int j = blockIdx.y, z = blockIdx.z;
  const int64_t n_ct = (g.d3 + TQ - 1) / TQ, n_rt = (g.R_out + C::TR - 1) / C::TR;
  const int64_t l = blockIdx.x, xcd = l % kXcds, jj = l / kXcds;
  const int64_t rt = (jj / n_ct) * kXcds + xcd, ct = jj % n_ct;
  if (rt >= n_rt) return;
  RnsTile t{g.Xr[z] + (size_t)j * g.KB * g.d3_pad * kKB, g.Dr[z] + (size_t)j * g.KB * g.R_pad * kKB,
            g.res + ((size_t)z * g.n_mod + j) * g.d3 * g.R_out, g.m[j], g.magic[j], g.KB, g.R_pad, g.d3_pad, g.n_db,
            g.row0, g.R_out, g.d3, rt * C::TR, ct * TQ};
  rns_tile<TQ>(t, lds);
}

// Persistent batched form: problem b's tiles are ordered (z, modulus, XCD-ordered tile), starting at
// its tile_begin; workgroups claim tiles in order from one counter per XCD (tile t = 8 j + xcd), as
// the digit form's batched kernel.
template <int TQ>
__global__ void __launch_bounds__(64 * RnsCfg<TQ>::NW) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_rns_batched(RnsBatchArgs a) {
  using C = RnsCfg<TQ>;
  __shared__ __attribute__((aligned(16))) int8_t lds[C::LDS];
  // this launch's problems and tiles (read on the device, so that a captured graph serves any batch)
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
    const int64_t n_ct = (d.d3 + TQ - 1) / TQ, n_rt = (d.R_out + C::TR - 1) / C::TR;
    const int64_t per_mod = (n_rt + kXcds - 1) / kXcds * kXcds * n_ct;
    const int64_t local = t - d.tile_begin;
    const int zj = (int)(local / per_mod);
    const int z = zj / a.n_mod, j = zj % a.n_mod;
    const int64_t l = local % per_mod, lj = l / kXcds;
    const int64_t rt = (lj / n_ct) * kXcds + l % kXcds, ct = lj % n_ct;
    if (rt >= n_rt) continue;
    RnsTile tl{d.Xd + ((size_t)z * a.n_mod + j) * a.KB * d.d3_pad * kKB,
               a.Dr + ((size_t)d.slot[z] * a.n_mod + j) * a.KB * a.R_pad * kKB,
               d.res + ((size_t)z * a.n_mod + j) * d.d3 * d.R_out, a.m[j], a.magic[j], a.KB, a.R_pad, d.d3_pad,
               d.n_db, d.row0, d.R_out, d.d3, rt * C::TR, ct * TQ};
    rns_tile<TQ>(tl, lds);
  }
}

int64_t rns_batched_tiles(int64_t d3, int64_t R_out, int nz, int n_mod, int tq) {
  const int64_t n_ct = (d3 + tq - 1) / tq, n_rt = (R_out + kRnsTileR - 1) / kRnsTileR;
  return (n_rt + kXcds - 1) / kXcds * kXcds * n_ct * nz * n_mod;
}

hipError_t launch_gemm_rns_batched(const RnsBatchArgs& a, int grid, int tq, hipStream_t s) {
  if (tq == 128)
    hipLaunchKernelGGL(k_gemm_rns_batched<128>, dim3((unsigned)grid), dim3(64 * RnsCfg<128>::NW), 0, s, a);
  else if (tq == 256)
    hipLaunchKernelGGL(k_gemm_rns_batched<256>, dim3((unsigned)grid), dim3(64 * RnsCfg<256>::NW), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// resident workgroups per CU: as many as the 160 KiB of LDS hold, at most two waves per SIMD
template <int TQ>
static int wgs_per_cu() {
  using C = RnsCfg<TQ>;
  const int by_lds = 160 * 1024 / C::LDS, by_waves = C::WPE * 4 / C::NW;
  const int w = by_lds < by_waves ? by_lds : by_waves;
  return w > 0 ? w : 1;
}
int rns_wgs_per_cu(int tq) { return tq == 128 ? wgs_per_cu<128>() : wgs_per_cu<256>(); }

// Query tile of the RNS contraction for a set of problems (d3, R_out, slots): the width whose
// padded work, weighted by its measured speed per column, is smaller (ties: 256).
int rns_tile_q(const int64_t* d3, const int64_t* R_out, const int* nz, int n) {
  double w128 = 0, w256 = 0;
  for (int i = 0; i < n; ++i) {
    const double rows = (double)((R_out[i] + kRnsTileR - 1) / kRnsTileR * kRnsTileR) * nz[i];
    w128 += rows * ((d3[i] + 127) / 128 * 128) * 1.09;
    w256 += rows * ((d3[i] + 255) / 256 * 256);
  }
  return w128 < w256 ? 128 : 256;
}

hipError_t launch_gemm_rns(const RnsGemmArgs& g, int tq, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  if ((tq != 128 && tq != 256) || g.d3_pad % tq != 0) return hipErrorInvalidValue;
  const int64_t n_ct = (g.d3 + tq - 1) / tq, n_rt = (g.R_out + kRnsTileR - 1) / kRnsTileR;
  const int64_t n_rt8 = (n_rt + kXcds - 1) / kXcds * kXcds;
  dim3 grid((unsigned)(n_rt8 * n_ct), (unsigned)g.n_mod, (unsigned)g.nz);
  if (tq == 128)
    hipLaunchKernelGGL(k_gemm_rns<128>, grid, dim3(64 * RnsCfg<128>::NW), 0, s, g);
  else
    hipLaunchKernelGGL(k_gemm_rns<256>, grid, dim3(64 * RnsCfg<256>::NW), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ CRT back to the prime
// Entry e of prime slot z: residues s_j = S mod m_j.  With y_j = s_j (M/m_j)^-1 mod m_j,
// S = sum_j y_j (M/m_j) - a M with a = round(sum_j y_j / m_j), since sum_j y_j (M/m_j) = S
// (mod M) and |S| <= M / 4 (the host chooses M >= 4 max |S|), so the fraction sum_j y_j / m_j
// - floor(...) = (S mod M) / M lies at least 1/4 away from 1/2 and single precision (error
// below 2^-19 over 16 terms) decides a exactly; then
// C = sum_j y_j ((M/m_j) mod q) - a (M mod q) mod q.
// Thread: 4 consecutive entries of one prime slot (blockIdx.y).
__global__ void __launch_bounds__(256) k_crt_rns(const uint8_t* res, int64_t n, RnsCrtArgs ra, uint64_t* C) {
  const int z = blockIdx.y;
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (e0 >= n) return;
  crt_quad(res + (size_t)z * ra.n * n, n, ra, z, C + (size_t)z * n, e0);
}

// CRT and rescale by p in one pass (single calls): per entry the residues of the special prime's
// slot (z = level) give cp, then each query prime's residue is reconstructed and rescaled,
// out[i][e] = (C_i - [cp] mod q_i) p^-1 mod q_i, so the contraction output C is never written.
// Thread: 4 consecutive entries (n a multiple of 4) or, otherwise, one entry.
__global__ void __launch_bounds__(256) k_crt_rescale_rns(const uint8_t* res, int64_t n, RnsCrtArgs ra,
                                                         RescaleArgs rs, uint64_t* out) {
  const int level = rs.level;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((n & 3) == 0) {
    const int64_t e0 = 4 * t;
    if (e0 >= n) return;
    uint64_t v[4];
    int64_t cp[4];
    crt_quad_vals(res + (size_t)level * ra.n * n, n, ra, level, e0, v);
#pragma unroll
    for (int b = 0; b < 4; ++b) cp[b] = centered(v[b], rs.p);
    for (int i = 0; i < level; ++i) {
      crt_quad_vals(res + (size_t)i * ra.n * n, n, ra, i, e0, v);
#pragma unroll
      for (int b = 0; b < 4; ++b) v[b] = rescale_value(v[b], cp[b], rs, i);
      reinterpret_cast<ulonglong2*>(out + (size_t)i * n + e0)[0] = make_ulonglong2(v[0], v[1]);
      reinterpret_cast<ulonglong2*>(out + (size_t)i * n + e0)[1] = make_ulonglong2(v[2], v[3]);
    }
  } else {
    const int64_t e = t;
    if (e >= n) return;
    const int64_t cp = centered(crt_entry(res + (size_t)level * ra.n * n + e, n, ra, level), rs.p);
    for (int i = 0; i < level; ++i)
      out[(size_t)i * n + e] = rescale_value(crt_entry(res + (size_t)i * ra.n * n + e, n, ra, i), cp, rs, i);
  }
}

hipError_t launch_crt_rescale_rns(const uint8_t* res, int64_t n, const RnsCrtArgs& ra, const RescaleArgs& rs,
                                  uint64_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t per = (n & 3) == 0 ? 4 : 1;
  const int64_t blocks = (n / per + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_crt_rescale_rns, dim3((unsigned)blocks), dim3(256), 0, s, res, n, ra, rs, out);
  return hipGetLastError();
}

hipError_t launch_crt_rns(const uint8_t* res, int nz, int64_t n, const RnsCrtArgs& ra, uint64_t* C,
                          hipStream_t s) {
  if (nz <= 0 || n <= 0) return hipSuccess;
  const int64_t blocks = (n + 4 * 256 - 1) / (4 * 256);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_crt_rns, dim3((unsigned)blocks, (unsigned)nz), dim3(256), 0, s, res, n, ra, C);
  return hipGetLastError();
}

}  // namespace hfe
