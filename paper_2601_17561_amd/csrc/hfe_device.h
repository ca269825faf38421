// Device-side element operations shared by the per-call and the grouped (batched) kernels:
// balanced int8 digit split, Garner mixed-radix reconstruction, the centered CRT lift of one
// query residue vector with its digit split, and the rescale of one output entry.
#pragma once

#include "hfe_internal.h"

namespace hfe {

// MFMA operand and result vectors: 16 int8 per lane (as 4 ints), 16 int32 per lane.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Contraction row r (0 .. N_DB + rows) -> database row: the A-part rows, then the shard's rows.
__device__ __forceinline__ int64_t src_row(int64_t r, int64_t n_db, int64_t row0) {
  return r < n_db ? r : r + row0;
}

// ------------------------------------------------------------------ digit split
// Centered residue x in (-q/2, q/2) -> 5 balanced base-256 digits d_t in [-128, 127]
// (|d_4| <= 8), x = sum_t d_t 256^t.
__device__ __forceinline__ void split5(int64_t x, int32_t d[kDigits]) {
#pragma unroll
  for (int t = 0; t < kDigits - 1; ++t) {
    const int32_t lo = (int32_t)((x + 128) & 255) - 128;
    d[t] = lo;
    x = (x - lo) >> 8;
  }
  d[kDigits - 1] = (int32_t)x;
}

// ------------------------------------------------------------------ Garner mixed radix
// Residues y_i mod q_i -> digits v_i with Y = v_0 + v_1 q_0 + v_2 q_0 q_1 + ..., computed as
// v_i = (y_i - sum_{j<i} v_j (q_0..q_{j-1} mod q_i)) * (q_0..q_{i-1})^-1 mod q_i.
// garner[i][j] = q_0..q_{j-1} mod q_i for j < i, garner[i][i] = (q_0..q_{i-1})^-1 mod q_i.
__device__ __forceinline__ void garner_digits(const uint64_t* y, int level,
                                              const uint64_t (*garner)[HFE_MAX_QPRIMES],
                                              const uint64_t* q, const uint64_t* mus, uint64_t* v) {
  for (int i = 0; i < level; ++i) {
    const uint64_t qi = q[i];
    const uint64_t mu = mus[i];
    uint64_t s = 0;
    for (int j = 0; j < i; ++j)
      s = add_mod(s, mul_mod(barrett64(v[j], qi, mu), garner[i][j], qi, mu), qi);
    v[i] = i == 0 ? y[0] : mul_mod(sub_mod(y[i], s, qi), garner[i][i], qi, mu);
  }
}

// Y > (Q - 1)/2, compared on mixed-radix digits from the most significant one.
__device__ __forceinline__ bool above_half(const uint64_t* v, const uint64_t* half, int level) {
  for (int i = level - 1; i >= 0; --i) {
    if (v[i] != half[i]) return v[i] > half[i];
  }
  return false;
}

// Query element (c, k) of XT ([level][d3][K]): the residues y_i of the lift L(x) = centered
// CRT value in (-Q/2, Q/2), and lp = L mod p.  Returns false for padding positions (c >= d3 or
// k >= K), where the lifted value is 0.
__device__ __forceinline__ bool lift_residues(const uint64_t* XT, int64_t d3, int64_t K, const LiftArgs& la,
                                              int64_t c, int64_t k, uint64_t* y, uint64_t& lp) {
  lp = 0;
  if (c >= d3 || k >= K) return false;
  for (int i = 0; i < la.level; ++i) y[i] = XT[((int64_t)i * d3 + c) * K + k];
  uint64_t v[HFE_MAX_QPRIMES];
  garner_digits(y, la.level, la.garner, la.q, la.mu, v);
  const uint64_t p = la.p;
  const uint64_t mup = la.mu_p;
  for (int i = 0; i < la.level; ++i)
    lp = add_mod(lp, mul_mod(barrett64(v[i], p, mup), la.mprod_p[i], p, mup), p);
  if (above_half(v, la.half_digits, la.level)) lp = sub_mod(lp, la.Q_mod_p, p);
  return true;
}

// Query element (c, k): writes Xp[c][k] = L mod p (if Xp) and the 5 digit planes of every prime
// of the level and p (if Xd), zero for padding positions.
__device__ __forceinline__ void lift_element(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                             int64_t d3_pad, const LiftArgs& la, uint64_t* Xp, int8_t* Xd,
                                             int64_t c, int64_t k) {
  uint64_t y[HFE_MAX_QPRIMES] = {};
  uint64_t lp;
  const bool valid = lift_residues(XT, d3, K, la, c, k, y, lp);
  if (valid && Xp) Xp[c * K + k] = lp;
  if (!Xd) return;
  const int64_t kb = k / kKB, kk = k % kKB;
  for (int z = 0; z <= la.level; ++z) {
    int64_t x = 0;
    if (valid) x = z < la.level ? centered(y[z], la.q[z]) : centered(lp, la.p);
    int32_t d[kDigits];
    split5(x, d);
#pragma unroll
    for (int t = 0; t < kDigits; ++t)
      Xd[((((int64_t)z * kDigits + t) * KB + kb) * d3_pad + c) * kKB + kk] = (int8_t)d[t];
  }
}

// ------------------------------------------------------------------ RNS form: small moduli
// x mod m for x < 2^24 and 2 <= m <= 256 with magic = ceil(2^32 / m): the quotient
// floor(x magic / 2^32) is exact because x (magic - 2^32 / m) / 2^32 < 2^-8 <= 1 / m.
__device__ __forceinline__ uint32_t mod_small(uint32_t x, uint32_t m, uint32_t magic) {
  return x - __umulhi(x, magic) * m;
}

// ------------------------------------------------------------------ balanced residues
// ceil(2^32 / m) for the moduli of kRnsMods.
__constant__ static uint32_t kRnsMagic[kRnsMaxMods] = {
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

// Query element (c, k) of the RNS form: for every prime of the level and p, the balanced residues
// of the centered lifted value modulo each small modulus, Xr[z][j][kb][c][kk] (zero in padding).
__device__ __forceinline__ void lift_element_rns(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                                 int64_t d3_pad, const LiftArgs& la, int n_mod, int8_t* Xr,
                                                 int64_t c, int64_t k) {
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

// CRT of one entry (see k_crt_rns): residues r[j n] mod m_j -> the exact centered sum mod the prime
// of database slot `slot`.
__device__ __forceinline__ uint64_t crt_entry(const uint8_t* r, int64_t n, const RnsCrtArgs& ra, int slot) {
  float frac = 0.f;
  uint64_t acc = 0;  // sum of y_j ((M/m_j) mod q) < 16 * 2^8 * 2^36
  for (int j = 0; j < ra.n; ++j) {
    const uint32_t y = mod_small((uint32_t)r[(size_t)j * n] * (uint32_t)ra.inv[j], (uint32_t)ra.m[j], ra.magic[j]);
    frac = fmaf((float)y, ra.rcp[j], frac);
    acc += (uint64_t)y * ra.Mj_mod_q[slot][j];
  }
  const uint64_t a = (uint64_t)(frac + 0.5f);
  const Mod md = ra.mod[slot];
  const uint64_t v = barrett64(acc, md.q, md.mu);
  return sub_mod(v, barrett64(a * ra.M_mod_q[slot], md.q, md.mu), md.q);
}

// Output entry e of a contraction (C[i] = residues mod q_i, Cp = residues mod p, n entries per
// prime): out[i][e] = (C[i][e] - centered(Cp[e]) mod q_i) * p^-1 mod q_i = RS_p of the CRT value.
// zstride: distance between the C entries of consecutive primes (n when C is [level + 1][n]).
__device__ __forceinline__ void rescale_element(const uint64_t* C, const uint64_t* Cp, int64_t n,
                                                const RescaleArgs& ra, uint64_t* out, int64_t e,
                                                int64_t zstride) {
  const int64_t cp = centered(Cp[e], ra.p);
  for (int i = 0; i < ra.level; ++i) {
    const Mod& m = ra.mod[i];
    const uint64_t r = from_signed(cp, m.q, m.mu);
    const uint64_t d = sub_mod(C[(int64_t)i * zstride + e], r, m.q);
    out[(int64_t)i * n + e] = mul_shoup(d, ra.pinv[i], ra.pinv_sh[i], m.q);
  }
}

}  // namespace hfe
