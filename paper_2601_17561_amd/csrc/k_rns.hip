// Small-modulus (RNS) int8 form of the modular contraction (Section 6.3: matrix products modulo a
// large modulus reduced to int8 products through RNS over small moduli).  For a prime q of the
// basis, C = D X mod q is recovered from the exact integer sum S = sum_k d_k x_k of centered
// residues: S mod m_j for n small pairwise coprime moduli m_j <= 256 (one int8 product each,
// int32 accumulation), then the CRT of those residues to S (the moduli's product exceeds 2 |S|),
// then S mod q.  One int8 product per modulus instead of 25 digit-pair products per prime.
#include "hfe_device.h"

namespace hfe {

// x mod m for x < 2^24 and 2 <= m <= 256 with magic = ceil(2^32 / m): the quotient
// floor(x magic / 2^32) is exact because x (magic - 2^32 / m) / 2^32 < 2^-8 <= 1 / m.
__device__ __forceinline__ uint32_t mod_small(uint32_t x, uint32_t m, uint32_t magic) {
  return x - __umulhi(x, magic) * m;
}

// ------------------------------------------------------------------ balanced residues
// ceil(2^32 / m) for the moduli of kRnsMods.
__constant__ uint32_t kRnsMagic[kRnsMaxMods] = {
    16777216u, 16843010u, 16976156u, 17111424u, 17388532u, 17821442u, 17970575u, 18433337u,
    18755316u, 18920561u, 19259944u, 20355296u, 21582751u, 21801865u, 22253717u, 22486740u};

// x (|x| < 2^40) -> x mod m_j in [-floor(m_j/2), ceil(m_j/2) - 1] for the modulus kRnsMods[j]:
// |x| = hi 2^24 + lo (hi < 2^16), |x| mod m = (hi (2^24 mod m) + lo) mod m with the argument
// split once more below 2^24.
__device__ __forceinline__ int32_t balanced_mod(int64_t x, int j) {
  const uint32_t m = (uint32_t)kRnsMods[j], mg = kRnsMagic[j];
  const uint64_t a = (uint64_t)(x < 0 ? -x : x);
  const uint32_t hi = (uint32_t)(a >> 24), lo = (uint32_t)(a & 0xFFFFFF);
  const uint32_t t24 = mod_small(mod_small(1u << 12, m, mg) * mod_small(1u << 12, m, mg), m, mg);
  const uint32_t hm = mod_small(mod_small(hi >> 8, m, mg) * mod_small(1u << 8, m, mg) + (hi & 255), m, mg);
  uint32_t r = mod_small(mod_small(hm * t24, m, mg) + mod_small(lo, m, mg), m, mg);
  if (x < 0 && r) r = m - r;
  return (int32_t)r >= ((int32_t)m + 1) / 2 ? (int32_t)r - (int32_t)m : (int32_t)r;
}

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
// Element (c, k): the lift of the query residues (as for the digit form), then for every prime
// of the level and p the balanced residues of the centered value modulo each small modulus:
// Xr[z][j][kb][c][kk], zero in the padding.
__global__ void __launch_bounds__(256) k_lift_rns(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                                  int64_t d3_pad, LiftArgs la, int n_mod, int8_t* Xr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (k >= KB * kKB) return;
  uint64_t y[HFE_MAX_QPRIMES] = {};
  uint64_t lp;
  const bool valid = lift_residues(XT, d3, K, la, c, k, y, lp);
  const int64_t kb = k / kKB, kk = k % kKB;
  for (int z = 0; z <= la.level; ++z) {
    int64_t x = 0;
    if (valid) x = z < la.level ? centered(y[z], la.q[z]) : centered(lp, la.p);
    for (int j = 0; j < n_mod; ++j)
      Xr[((((int64_t)z * n_mod + j) * KB + kb) * d3_pad + c) * kKB + kk] = (int8_t)balanced_mod(x, j);
  }
}

hipError_t launch_lift_rns(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                           const LiftArgs& la, int n_mod, int8_t* Xr, hipStream_t s) {
  dim3 grid((unsigned)((KB * kKB + 255) / 256), (unsigned)d3_pad);
  hipLaunchKernelGGL(k_lift_rns, grid, dim3(256), 0, s, XT, d3, K, KB, d3_pad, la, n_mod, Xr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ contraction per modulus
// Workgroup: 4 x 2 waves (two per SIMD) on 256 database rows x 256 query columns of one (prime,
// modulus); wave (wq, wr) owns 64 query columns x 128 rows as 2 x 4 blocks of 32 x 32 with one
// int32 accumulator each (v_mfma_i32_32x32x32_i8), so each fragment read from LDS feeds 2 or 4
// MFMAs.  One 64-byte K-block of both operands per LDS stage (32 KiB), three stages fed by direct
// global-to-LDS loads (same row swizzle as the digit form's DMA tiles), so two K-blocks are in
// flight while one is multiplied.  Exactness: |S| over the K-range <= K * 128 * 128 < 2^31 for
// K < 2^17 (checked by the host).
constexpr int kRnsWQB = 2, kRnsWRB = 4, kRnsNQ = kRnsTileQ / 64, kRnsNR = kRnsTileR / 128;
constexpr int kRnsNW = kRnsNQ * kRnsNR, kRnsStages = 3;
constexpr int kRnsPA = kRnsTileQ * kKB, kRnsPB = kRnsTileR * kKB, kRnsStage = kRnsPA + kRnsPB;
constexpr int kRnsLA = kRnsTileQ / 16 / kRnsNW, kRnsLB = kRnsTileR / 16 / kRnsNW;  // 2 + 2 loads per wave

__device__ __forceinline__ void dma16_rns(const int8_t* g, uint32_t lds_addr) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
               : "memory", "m0");
}

__global__ void __launch_bounds__(64 * kRnsNW) __attribute__((amdgpu_waves_per_eu(2, 2))) k_gemm_rns(RnsGemmArgs g) {
  static_assert(kRnsNW == 8 && kRnsLA + kRnsLB == 4, "the vmcnt below assumes 4 loads per wave per K-block");
  __shared__ __attribute__((aligned(16))) int8_t lds[kRnsStages * kRnsStage];
  const int j = blockIdx.y, z = blockIdx.z;
  const int64_t n_ct = (g.d3 + kRnsTileQ - 1) / kRnsTileQ, n_rt = (g.R_out + kRnsTileR - 1) / kRnsTileR;
  const int64_t l = blockIdx.x, xcd = l % kXcds, jj = l / kXcds;
  const int64_t rt = (jj / n_ct) * kXcds + xcd, ct = jj % n_ct;
  if (rt >= n_rt) return;
  const int64_t r0 = rt * kRnsTileR, c0 = ct * kRnsTileQ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wq = wave % kRnsNQ, wr = wave / kRnsNQ;
  const int8_t* X = g.Xr[z] + (size_t)j * g.KB * g.d3_pad * kKB;
  const int8_t* D = g.Dr[z] + (size_t)j * g.KB * g.R_pad * kKB;
  const size_t stepA = (size_t)g.d3_pad * kKB, stepB = (size_t)g.R_pad * kKB;
  // load i of a wave fills tile rows 16 (wave + 4 i) .. + 15 (lane l: row + l / 4, stored chunk
  // l % 4 holding logical chunk (l % 4) ^ ((row >> 2) & 3))
  const int ld_row = 16 * wave + (lane >> 2);
  const int ld_chunk = ((lane & 3) ^ ((ld_row >> 2) & 3)) * 16;
  const int8_t* gA[kRnsLA];
  const int8_t* gB[kRnsLB];
#pragma unroll
  for (int i = 0; i < kRnsLA; ++i) gA[i] = X + (size_t)(c0 + ld_row + 16 * kRnsNW * i) * kKB + ld_chunk;
#pragma unroll
  for (int i = 0; i < kRnsLB; ++i)
    gB[i] = D + (size_t)src_row(r0 + ld_row + 16 * kRnsNW * i, g.n_db, g.row0) * kKB + ld_chunk;
  const uint32_t lds0 = (uint32_t)(uintptr_t)lds + wave * 16 * kKB;
  auto issue = [&](int stage, int64_t kb) {
    const uint32_t base = lds0 + stage * kRnsStage;
#pragma unroll
    for (int i = 0; i < kRnsLA; ++i) dma16_rns(gA[i] + kb * stepA, base + 16 * kRnsNW * i * kKB);
#pragma unroll
    for (int i = 0; i < kRnsLB; ++i) dma16_rns(gB[i] + kb * stepB, base + kRnsPA + 16 * kRnsNW * i * kKB);
  };
  const int sw = ((lane & 31) >> 2) & 3, cl = lane >> 5;
  const int offA = (wq * 32 * kRnsWQB + (lane & 31)) * kKB;
  const int offB = kRnsPA + (wr * 32 * kRnsWRB + (lane & 31)) * kKB;
  v16i acc[kRnsWQB][kRnsWRB];
#pragma unroll
  for (int a = 0; a < kRnsWQB; ++a)
#pragma unroll
    for (int b = 0; b < kRnsWRB; ++b) acc[a][b] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t KB = g.KB;
  auto clamp = [&](int64_t i) { return i < KB ? i : KB - 1; };
  issue(0, clamp(0));
  issue(1, clamp(1));
  for (int64_t i = 0; i < KB; ++i) {
    // block i complete for this wave (block i + 1 may still fly), then for all waves; all waves
    // are done reading the stage that block i + 2 overwrites
    asm volatile("s_waitcnt vmcnt(4) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    issue((int)((i + 2) % kRnsStages), clamp(i + 2));
    const int8_t* S = lds + (int)(i % kRnsStages) * kRnsStage;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int chunk = ((cl + 2 * h) ^ sw) << 4;
      v4i fa[kRnsWQB], fb[kRnsWRB];
#pragma unroll
      for (int a = 0; a < kRnsWQB; ++a) fa[a] = *reinterpret_cast<const v4i*>(S + offA + a * 32 * kKB + chunk);
#pragma unroll
      for (int b = 0; b < kRnsWRB; ++b) fb[b] = *reinterpret_cast<const v4i*>(S + offB + b * 32 * kKB + chunk);
#pragma unroll
      for (int a = 0; a < kRnsWQB; ++a)
#pragma unroll
        for (int b = 0; b < kRnsWRB; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  }
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  // epilogue: S mod m_j in [0, m_j) -> res[z][j][c][r]; 32 x 32 result layout as in the digit
  // form (lane l, element e: query column 8 (e / 4) + 4 (l / 32) + e % 4, row l % 32)
  const int32_t m = g.m[j];
  const uint32_t magic = g.magic[j];
  // |acc| < 2^31: u = acc + 2^31 = hi 2^17 + lo (hi < 2^15), and
  // acc mod m = (hi (2^17 mod m) + lo + (m - 2^31 mod m)) mod m with the argument below 2^24
  const uint32_t t16 = mod_small(1u << 16, (uint32_t)m, magic), t17 = mod_small(1u << 17, (uint32_t)m, magic);
  const uint32_t off = (uint32_t)m - mod_small(mod_small(1u << 15, (uint32_t)m, magic) * t16, (uint32_t)m, magic);
  uint16_t* res = g.res + ((size_t)z * g.n_mod + j) * g.d3 * g.R_out;
#pragma unroll
  for (int b = 0; b < kRnsWRB; ++b) {
    const int64_t r = r0 + wr * 32 * kRnsWRB + b * 32 + (lane & 31);
    if (r >= g.R_out) continue;
#pragma unroll
    for (int a = 0; a < kRnsWQB; ++a)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t c = c0 + wq * 32 * kRnsWQB + a * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (c >= g.d3) continue;
        const uint32_t u = (uint32_t)acc[a][b][e] + 0x80000000u;  // acc + 2^31 >= 0
        const uint32_t v = mod_small((u >> 17) * t17 + (u & 0x1FFFF) + off, (uint32_t)m, magic);
        res[c * g.R_out + r] = (uint16_t)v;
      }
  }
}

hipError_t launch_gemm_rns(const RnsGemmArgs& g, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  if (g.d3_pad % kRnsTileQ != 0) return hipErrorInvalidValue;
  const int64_t n_ct = (g.d3 + kRnsTileQ - 1) / kRnsTileQ, n_rt = (g.R_out + kRnsTileR - 1) / kRnsTileR;
  const int64_t n_rt8 = (n_rt + kXcds - 1) / kXcds * kXcds;
  dim3 grid((unsigned)(n_rt8 * n_ct), (unsigned)g.n_mod, (unsigned)g.nz);
  hipLaunchKernelGGL(k_gemm_rns, grid, dim3(64 * kRnsNW), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ CRT back to the prime
// Entry e of prime slot z: residues s_j = S mod m_j.  With y_j = s_j (M/m_j)^-1 mod m_j,
// S = sum_j y_j (M/m_j) - a M with a = round(sum_j y_j / m_j), since sum_j y_j (M/m_j) = S
// (mod M) and |S| <= M / 4 (the host chooses M >= 4 max |S|), so the fraction sum_j y_j / m_j
// - floor(...) = (S mod M) / M lies at least 1/4 away from 1/2 and single precision (error
// below 2^-19 over 16 terms) decides a exactly; then
// C = sum_j y_j ((M/m_j) mod q) - a (M mod q) mod q.
__global__ void __launch_bounds__(256) k_crt_rns(const uint16_t* res, int nz, int64_t n, RnsCrtArgs ra, uint64_t* C) {
  const int64_t total = (int64_t)nz * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(t / n);
    const int64_t e = t - (int64_t)z * n;
    const uint16_t* r = res + (size_t)z * ra.n * n + e;
    float frac = 0.f;
    uint64_t acc = 0;  // sum of y_j ((M/m_j) mod q) < 16 * 2^8 * 2^36
    for (int j = 0; j < ra.n; ++j) {
      const uint32_t y = mod_small((uint32_t)r[(size_t)j * n] * (uint32_t)ra.inv[j], (uint32_t)ra.m[j], ra.magic[j]);
      frac = fmaf((float)y, ra.rcp[j], frac);
      acc += (uint64_t)y * ra.Mj_mod_q[z][j];
    }
    const uint64_t a = (uint64_t)(frac + 0.5f);
    const Mod md = ra.mod[z];
    uint64_t v = barrett64(acc, md.q, md.mu);
    v = sub_mod(v, barrett64(a * ra.M_mod_q[z], md.q, md.mu), md.q);
    C[(size_t)z * n + e] = v;
  }
}

hipError_t launch_crt_rns(const uint16_t* res, int nz, int64_t n, const RnsCrtArgs& ra, uint64_t* C,
                          hipStream_t s) {
  const int64_t total = (int64_t)nz * n;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_crt_rns, dim3((unsigned)blocks), dim3(256), 0, s, res, nz, n, ra, C);
  return hipGetLastError();
}

}  // namespace hfe
