// The CCMM over the paper's own modulus chain (Section 6.3, "Fast PPMM using int8 cuBLAS"): the
// ciphertext modulus is a product of squares n^2 of primes 127 <= n <= 253, so a product modulo the
// modulus is a product modulo each n^2, and that is three int8 products of the digits M + n M'
// (M N + n (M N' + M' N) mod n^2) with no integer to rebuild.  The contraction itself is the n^2
// kernel of k_p2.hip (one base per modulus); this file holds the parts around it: the database split
// into M, M' per modulus, the query lift from Q = prod m_j to the special moduli m'_s of P, and the
// rescale by the composite P, RS_P(x) = floor(x / P + 1/2) mod Q (Section 2.2.4; P odd, no ties).
#include "hfe_device.h"

namespace hfe {

ChainBase chain_base(int32_t n) {
  ChainBase b;
  b.n = n;
  b.m = n * n;
  b.magic_n = (uint32_t)(((1ull << 32) + (uint64_t)n - 1) / (uint64_t)n);
  b.rcp_n = 1.0 / (double)n;
  b.rcp_m = 1.0 / (double)b.m;
  return b;
}

// ------------------------------------------------------------------ database split
// Thread (row r, K-block kb): 64 residues Dt[k][r] mod n^2, centered -> one 64-byte row of M (plane 0)
// and one of M' (plane 1).
__global__ void __launch_bounds__(256) k_chain_split_db(const uint64_t* Dt, int64_t K, int64_t R, int64_t KB,
                                                        int64_t R_pad, ChainBase b, int8_t* planes) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kb = blockIdx.y;
  if (r >= R_pad) return;
  uint4* d0 = reinterpret_cast<uint4*>(planes + ((int64_t)kb * R_pad + r) * kKB);
  uint4* d1 = reinterpret_cast<uint4*>(planes + (((int64_t)KB + kb) * R_pad + r) * kKB);
#pragma unroll
  for (int i = 0; i < kKB / 16; ++i) {
    uint32_t w0[4], w1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      uint32_t v0 = 0, v1 = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t k = kb * kKB + 16 * i + 4 * t + e;
        const int64_t x = (r < R && k < K) ? centered(Dt[k * R + r], (uint64_t)b.m) : 0;
        int32_t M, Mp;
        p2_digits_by(x, b.n, b.m, b.magic_n, b.rcp_m, M, Mp);
        v0 |= ((uint32_t)M & 255u) << (8 * e);
        v1 |= ((uint32_t)Mp & 255u) << (8 * e);
      }
      w0[t] = v0;
      w1[t] = v1;
    }
    d0[i] = make_uint4(w0[0], w0[1], w0[2], w0[3]);
    d1[i] = make_uint4(w1[0], w1[1], w1[2], w1[3]);
  }
}

hipError_t launch_chain_split_db(const uint64_t* Dt, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                                 const ChainBase& b, int8_t* planes, hipStream_t s) {
  dim3 grid((unsigned)((R_pad + 255) / 256), (unsigned)KB);
  hipLaunchKernelGGL(k_chain_split_db, grid, dim3(256), 0, s, Dt, K, R, KB, R_pad, b, planes);
  return hipGetLastError();
}

// ------------------------------------------------------------------ query lift
// Element (c, k) by lane k mod 4 of a quad holding k - k mod 4 .. + 3 of column c (whole quads
// active): the residues y_j mod m_j of the query; their mixed-radix (Garner) digits give the
// centered lift L in (-Q/2, Q/2), taken mod each special modulus m'_s as sum_i v_i (m_0..m_{i-1}
// mod m'_s), minus Q mod m'_s when L is negative (the digits above (Q - 1)/2).  Every slot's
// centered value becomes its digits M, M', stored by the quad's first lane as one 4-byte word per
// plane: Xq[slot][t][kb][c][kk], zero in the padding (c >= d3 or k >= K).
__global__ void __launch_bounds__(256) k_chain_lift(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                                    int64_t d3_pad, ChainLiftArgs la, int8_t* Xq) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= KB * kKB) return;
  const int64_t c = blockIdx.y;
  const bool valid = c < d3 && k < K;
  // every modulus is n^2 <= 2^16: Garner's digits and the lift to the special moduli in 32-bit products
  uint32_t y[HFE_MAX_QPRIMES] = {}, v[HFE_MAX_QPRIMES] = {};
  uint32_t lp[kChainMaxP] = {};
  if (valid) {
#pragma unroll
    for (int i = 0; i < HFE_MAX_QPRIMES; ++i)
      if (i < la.level) y[i] = (uint32_t)XT[((int64_t)i * d3 + c) * K + k];
    garner_digits_u16(y, la.level, la.garner, la.q, la.qmagic, v);
    bool neg = false, decided = false;  // the lift above (Q - 1) / 2, compared on the digits from the top
#pragma unroll
    for (int i = HFE_MAX_QPRIMES - 1; i >= 0; --i)
      if (i < la.level && !decided && v[i] != (uint32_t)la.half_digits[i]) {
        neg = v[i] > (uint32_t)la.half_digits[i];
        decided = true;
      }
#pragma unroll
    for (int s = 0; s < kChainMaxP; ++s) {
      if (s >= la.np) break;
      const uint32_t pm = (uint32_t)la.pm[s], mg = la.pmagic[s];
      uint32_t acc = 0;
#pragma unroll
      for (int i = 0; i < HFE_MAX_QPRIMES; ++i)
        if (i < la.level) {
          acc += mulmod_u16(mod_u32(v[i], pm, mg), (uint32_t)la.mprod[s][i], pm, mg);
          acc = acc >= pm ? acc - pm : acc;
        }
      const uint32_t qm = (uint32_t)la.Q_mod[s];
      lp[s] = neg ? (acc >= qm ? acc - qm : acc + pm - qm) : acc;
    }
  }
  const bool writer = (threadIdx.x & 3) == 0;
  const int64_t kb = k / kKB, kk = k % kKB - (k & 3);
  const int64_t pstride = KB * d3_pad * kKB / 4;  // words between consecutive planes
  auto emit = [&](int slot, int64_t x) {
    const ChainBase& b = la.base[slot];
    int32_t M, Mp;
    p2_digits_by(x, b.n, b.m, b.magic_n, b.rcp_m, M, Mp);
    const uint32_t w0 = quad_word((uint32_t)M), w1 = quad_word((uint32_t)Mp);
    uint32_t* row = reinterpret_cast<uint32_t*>(Xq + (((int64_t)(2 * slot) * KB + kb) * d3_pad + c) * kKB + kk);
    if (writer) {
      row[0] = w0;
      row[pstride] = w1;
    }
  };
#pragma unroll
  for (int s = 0; s < kChainMaxP; ++s)
    if (s < la.np) emit(s, valid ? centered(lp[s], la.pm[s]) : 0);
#pragma unroll
  for (int j = 0; j < HFE_MAX_QPRIMES; ++j)
    if (j < la.level) emit(la.np + j, valid ? centered(y[j], la.q[j]) : 0);
}

hipError_t launch_chain_lift(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                             const ChainLiftArgs& la, int8_t* Xq, hipStream_t s) {
  if (la.level < 1 || la.level > HFE_MAX_QPRIMES || la.np < 1 || la.np > kChainMaxP) return hipErrorInvalidValue;
  dim3 grid((unsigned)((KB * kKB + 255) / 256), (unsigned)d3_pad);
  hipLaunchKernelGGL(k_chain_lift, grid, dim3(256), 0, s, XT, d3, K, KB, d3_pad, la, Xq);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rescale by P
// Entry e: the residues r_s = x mod m'_s give, by Garner's mixed radix, x mod P as an integer X < P
// (below 2^48), and its centered form x_P in (-P/2, P/2).  Then for each query modulus
// RS_P(x) mod m_j = (x mod m_j - x_P) P^-1 mod m_j, exact because x - x_P is a multiple of P, and
// equal to floor(x / P + 1/2) because x_P is the centered remainder (P odd).
__global__ void __launch_bounds__(256) k_chain_rescale(const uint16_t* res, int64_t n, ChainRescaleArgs ra,
                                                       uint64_t* out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t X = 0, pre = 1;
#pragma unroll
    for (int s = 0; s < kChainMaxP; ++s) {
      if (s >= ra.np) break;
      const uint64_t pm = ra.pm[s], pmu = ra.pmu[s];
      const uint64_t r = res[(int64_t)s * n + e];
      const uint64_t d = mulmod_u16((uint32_t)sub_mod(r, barrett64(X, pm, pmu), pm), (uint32_t)ra.pinv[s],
                                    (uint32_t)pm, ra.pmagic[s]);
      X += d * pre;
      pre *= pm;
    }
    const int64_t xp = X > (ra.P >> 1) ? (int64_t)X - (int64_t)ra.P : (int64_t)X;
#pragma unroll
    for (int j = 0; j < HFE_MAX_QPRIMES; ++j) {
      if (j >= ra.level) break;
      const Mod& M = ra.mod[j];
      const uint64_t cj = res[(int64_t)(ra.np + j) * n + e];
      out[(int64_t)j * n + e] = mulmod_u16((uint32_t)sub_mod(cj, from_signed(xp, M.q, M.mu), M.q),
                                           (uint32_t)ra.Pinv[j], (uint32_t)M.q, ra.qmagic[j]);
    }
  }
}

hipError_t launch_chain_rescale(const uint16_t* res, int64_t n, const ChainRescaleArgs& ra, uint64_t* out,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (ra.level < 1 || ra.level > HFE_MAX_QPRIMES || ra.np < 1 || ra.np > kChainMaxP) return hipErrorInvalidValue;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_chain_rescale, dim3((unsigned)blocks), dim3(256), 0, s, res, n, ra, out);
  return hipGetLastError();
}

// The contraction residues in the export order of hfe_ccmm_product (the level's query moduli, then the
// special ones): C[i][e] = res[slot(i)][e] with slot(i) = np + i for i < level, i - level after.
__global__ void k_chain_widen(const uint16_t* res, int64_t n, int level, int np, uint64_t* C) {
  const int i = blockIdx.y;
  const int slot = i < level ? np + i : i - level;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    C[(int64_t)i * n + e] = res[(int64_t)slot * n + e];
}

hipError_t launch_chain_widen(const uint16_t* res, int64_t n, int level, int np, uint64_t* C, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_chain_widen, dim3((unsigned)blocks, (unsigned)(level + np)), dim3(256), 0, s, res, n, level, np,
                     C);
  return hipGetLastError();
}

}  // namespace hfe
