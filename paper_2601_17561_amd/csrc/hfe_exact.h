// Exact integer results reached through floating point or multiply-high quotients.
//
// Every helper here returns an exact integer (a residue, a quotient, a balanced digit) although part
// of its arithmetic runs in fp64, fp32 or as a 32-bit multiply-high by a precomputed reciprocal.
// Each comment states the operand range for which the result is exact.  The helpers are host and
// device functions: the kernels call them, and a host build of the same code is checked against
// exact integer arithmetic by the CPU tests (tests/native/exact_check.cpp).
#pragma once

#include <math.h>
#include <stdint.h>

#include "hfe_math.h"

namespace hfe {

// ------------------------------------------------------------------ fp64 residues mod q < 2^36
// Residues as doubles holding exact integers in [0, q).
// a w mod q for a, w in [0, q), q < 2^36, qinv = RN(1/q): hi = RN(a w) is an integer and
// lo = a w - hi (|lo| <= 2^18) is exact from one fused multiply-add; t = floor(hi qinv) is within one
// of floor(a w / q) (relative error below 3 2^-53 on a quotient below 2^36); hi - t q is an integer
// below 2^38 in magnitude, so the second fused multiply-add is exact, and so is adding lo.  The result
// lies in (-q, 2q) and one conditional correction each way brings it to [0, q).
HFE_HD double mulmod_d(double a, double w, double q, double qinv) {
#pragma clang fp contract(off)
  const double hi = a * w;
  const double lo = __builtin_fma(a, w, -hi);
  const double t = __builtin_floor(hi * qinv);
  double r = __builtin_fma(-t, q, hi) + lo;
  r = r < 0.0 ? r + q : r;
  return r >= q ? r - q : r;
}
// Signed transforms (the FormatSwitch kernels): values are integers held as doubles, congruent to
// the residues and bounded in magnitude, never corrected inside a transform.
// a w mod q as a centered representative, for integers |a| <= 16q and w in [0, q), q < 2^36:
// P = a w is below 2^76 in magnitude, hi = RN(P) an integer with |hi - P| <= 2^22, lo = P - hi exact
// from one fused multiply-add; u = hi qinv is within 2^-11 of P / q (|d| / q <= 2^-13 plus a relative
// error below 2^-52 on a quotient below 2^40), so t = rint(u) is within 1/2 + 2^-11 of P / q and
// P - t q = (hi - t q) + lo is an exact integer of magnitude at most (1/2 + 2^-11) q.
HFE_HD double mulmod_c_d(double a, double w, double q, double qinv) {
#pragma clang fp contract(off)
  const double hi = a * w;
  const double lo = __builtin_fma(a, w, -hi);
  const double t = __builtin_rint(hi * qinv);
  return __builtin_fma(-t, q, hi) + lo;
}
// x - q rint(x / q) for an integer |x| < 2^47: exact, of magnitude at most (1/2 + 2^-11) q.
HFE_HD double reduce_c_d(double x, double q, double qinv) {
#pragma clang fp contract(off)
  return __builtin_fma(-__builtin_rint(x * qinv), q, x);
}
// A centered value (|x| < q) to its residue in [0, q).
HFE_HD double residue_of_c(double x, double q) { return x < 0.0 ? x + q : x; }
// Cooley-Tukey butterfly on signed values: (X, Y) -> (X + W Y, X - W Y) with W Y centered.  Each
// stage adds at most (1/2 + 2^-11) q to the magnitude: inputs below 2q stay below 9.1q over 14 stages.
HFE_HD void ct_butterfly_c(double& X, double& Y, double W, double q, double qinv) {
  const double t = mulmod_c_d(Y, W, q, qinv);
  const double x = X;
  X = x + t;
  Y = x - t;
}
HFE_HD double addmod_d(double a, double b, double q) {
  const double s = a + b;  // exact below 2^37
  return s >= q ? s - q : s;
}
HFE_HD double submod_d(double a, double b, double q) {
  const double d = a - b;
  return d < 0.0 ? d + q : d;
}

// ------------------------------------------------------------------ small moduli m <= 256
// High 32 bits of a 32 x 32 product (one v_mul_hi_u32 on the device).
HFE_HD uint32_t umulhi32(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }

// x mod m for x < 2^24 and 2 <= m <= 256 with magic = ceil(2^32 / m): the quotient
// floor(x magic / 2^32) is exact because x (magic - 2^32 / m) / 2^32 < 2^24 / 2^32 < 1 / m.
// (Also exact for x < 2^17 and any m < 2^15: x (magic - 2^32/m) < 2^17 < 2^32 / m.)
HFE_HD uint32_t mod_small(uint32_t x, uint32_t m, uint32_t magic) { return x - umulhi32(x, magic) * m; }

// x mod m for any x < 2^32 and 2 <= m <= 2^16, magic = ceil(2^32 / m): x magic / 2^32 exceeds x / m by
// x (magic - 2^32 / m) / 2^32 < 1, so the estimate is the quotient or one more; one correction.
HFE_HD uint32_t mod_u32(uint32_t x, uint32_t m, uint32_t magic) {
  const uint32_t qe = umulhi32(x, magic);
  const int64_t r = (int64_t)x - (int64_t)qe * (int64_t)m;
  return (uint32_t)(r < 0 ? r + m : r);
}
// a b mod m for a, b < m <= 2^16 (the n^2 moduli of the modulus chain): a b < 2^32.
HFE_HD uint32_t mulmod_u16(uint32_t a, uint32_t b, uint32_t m, uint32_t magic) { return mod_u32(a * b, m, magic); }
HFE_HD uint32_t magic_u32(uint32_t m) { return (uint32_t)(((1ull << 32) + m - 1) / m); }

// x mod m in [0, m) for |x| < 2^48 and 2 <= m < 2^24, rcp = RN(1 / m): x rcp differs from x / m by
// less than 2^-4, so floor(x rcp) is the quotient or one off, fixed by one step.
HFE_HD int64_t mod_f64(int64_t x, int64_t m, double rcp) {
  int64_t r = x - (int64_t)__builtin_floor((double)x * rcp) * m;
  if (r < 0)
    r += m;
  else if (r >= m)
    r -= m;
  return r;
}

// ------------------------------------------------------------------ RNS form: moduli and residues
// Pairwise coprime moduli <= 256 (balanced residues fit int8), largest product first: 2^8,
// 3*5*17, 11*23, 251, 13*19, then primes.  A database uses the shortest prefix whose product is at
// least four times the largest exact contraction sum (Section 6.3, RNS over small moduli).
constexpr int kRnsMaxMods = 16;
constexpr int32_t kRnsMods[kRnsMaxMods] = {256, 255, 253, 251, 247, 241, 239, 233,
                                           229, 227, 223, 211, 199, 197, 193, 191};

// Per small modulus m_j: m_j, ceil(2^32 / m_j) and 2^24 mod m_j.
struct RnsModConsts {
  uint32_t m[kRnsMaxMods], magic[kRnsMaxMods], t24[kRnsMaxMods];
};
constexpr RnsModConsts make_rns_mod_consts() {
  RnsModConsts c{};
  for (int j = 0; j < kRnsMaxMods; ++j) {
    const uint64_t m = (uint64_t)kRnsMods[j];
    c.m[j] = (uint32_t)m;
    c.magic[j] = (uint32_t)(((1ull << 32) + m - 1) / m);
    c.t24[j] = (uint32_t)((1ull << 24) % m);
  }
  return c;
}

// x (|x| < 2^40) -> x mod m in [-floor(m/2), ceil(m/2) - 1]: |x| = hi 2^24 + lo (hi < 2^16), and
// |x| mod m = (hi (2^24 mod m) + (lo mod m)) mod m, whose argument is at most
// (2^16 - 1)(m - 1) + m - 1 < 2^24.
HFE_HD int32_t balanced_mod_by(int64_t x, uint32_t m, uint32_t magic, uint32_t t24) {
  const uint64_t a = (uint64_t)(x < 0 ? -x : x);
  const uint32_t hi = (uint32_t)(a >> 24), lo = (uint32_t)(a & 0xFFFFFF);
  uint32_t r = mod_small(hi * t24 + mod_small(lo, m, magic), m, magic);
  if (x < 0 && r) r = m - r;
  return (int32_t)r >= ((int32_t)m + 1) / 2 ? (int32_t)r - (int32_t)m : (int32_t)r;
}

// The contraction epilogue of the RNS form: an int32 sum S (|S| < 2^31) -> S mod m in [0, m).
// u = S + 2^31 = hi 2^17 + lo (hi < 2^15, lo < 2^17), and S mod m = (hi (2^17 mod m) + lo + off) mod m
// with off = m - (2^31 mod m); the argument is below 2^15 2^8 + 2^17 + 2^8 < 2^24.
struct RnsAccConsts {
  uint32_t t17, off;
};
HFE_HD RnsAccConsts rns_acc_consts(uint32_t m, uint32_t magic) {
  const uint32_t t16 = mod_small(1u << 16, m, magic), t17 = mod_small(1u << 17, m, magic);
  RnsAccConsts c;
  c.t17 = t17;
  c.off = m - mod_small(mod_small(1u << 15, m, magic) * t16, m, magic);
  return c;
}
HFE_HD uint32_t rns_acc_mod(int32_t s, uint32_t m, uint32_t magic, RnsAccConsts c) {
  const uint32_t u = (uint32_t)s + 0x80000000u;
  return mod_small((u >> 17) * c.t17 + (u & 0x1FFFF) + c.off, m, magic);
}

// ------------------------------------------------------------------ n^2 form: bases and digits
// Bases n of the n^2 form (Section 6.3, a matrix modulo n^2 as M + n M'): primes 127 <= n <= 253,
// largest first.  A database uses the shortest prefix whose squares' product is at least four
// times the largest exact contraction sum; at most 8 (the product stays below 2^128).
constexpr int kP2MaxBases = 8;
constexpr int32_t kP2Bases[kP2MaxBases] = {251, 241, 239, 233, 229, 227, 223, 211};

// Per base n_j: n_j, n_j^2, their reciprocals and ceil(2^32 / n_j).
struct P2BaseConsts {
  int32_t n[kP2MaxBases], m[kP2MaxBases];
  uint32_t magic_n[kP2MaxBases];
  double rcp_n[kP2MaxBases], rcp_m[kP2MaxBases];
};
constexpr P2BaseConsts make_p2_base_consts() {
  P2BaseConsts c{};
  for (int j = 0; j < kP2MaxBases; ++j) {
    c.n[j] = kP2Bases[j];
    c.m[j] = kP2Bases[j] * kP2Bases[j];
    c.magic_n[j] = (uint32_t)(((1ull << 32) + (uint64_t)c.n[j] - 1) / (uint64_t)c.n[j]);
    c.rcp_n[j] = 1.0 / (double)c.n[j];
    c.rcp_m[j] = 1.0 / (double)c.m[j];
  }
  return c;
}

// Centered x (|x| < 2^48) -> (M, M') with x = M + n M' (mod n^2), both in [-(n-1)/2, (n-1)/2]:
// r = x mod n^2, M = the balanced residue of r mod n, M' = the balanced residue of (r - M) / n (an
// integer in [0, n]) mod n.  After the first step everything is below 2^17, where the multiply-high
// quotient by ceil(2^32 / n) is exact (mod_small).
HFE_HD void p2_digits_by(int64_t x, int32_t n, int32_t nsq, uint32_t magic, double rcp_nsq, int32_t& M,
                         int32_t& Mp) {
  const int32_t h = (n - 1) / 2;
  const uint32_t r = (uint32_t)mod_f64(x, nsq, rcp_nsq);
  M = (int32_t)mod_small(r, (uint32_t)n, magic);
  if (M > h) M -= n;
  const uint32_t rm = (uint32_t)((int32_t)r - M);  // a multiple of n in [0, n^2 + h]
  int32_t t = (int32_t)umulhi32(rm, magic);         // (r - M) / n, exact
  if (t == n) t = 0;
  Mp = t > h ? t - n : t;
}

// The contraction epilogue of the n^2 form: from the int32 sums G0 = sum M N and G1 = sum (M N' + M' N),
// S mod n^2 = (G0 mod n^2 + n (G1 mod n)) mod n^2.
HFE_HD uint32_t p2_acc_mod(int32_t g0, int32_t g1, int32_t n, int32_t nsq, double rcp_n, double rcp_nsq) {
  int32_t v = (int32_t)mod_f64(g0, nsq, rcp_nsq) + n * (int32_t)mod_f64(g1, n, rcp_n);
  return (uint32_t)(v >= nsq ? v - nsq : v);
}

// ------------------------------------------------------------------ CRT from small moduli
// The exact centered sum S (|S| <= M / 4, M = the product of the moduli m_j) from its residues
// s_j = S mod m_j, reduced mod a prime q (the fractional-sum form of the CRT; Kawamura et al. 2000):
// with y_j = s_j (M/m_j)^-1 mod m_j, S = sum_j y_j (M/m_j) - a M where a = round(sum_j y_j / m_j).
// The exact fraction sum_j y_j / m_j = a + S / M lies within 1/4 of the integer a; the fp32 sum of at
// most 16 terms y_j RN(1/m_j) (each below 2^8 with a relative error of 2^-24 in the reciprocal, and
// one rounding per fused multiply-add of a value below 16) is off by far less than 1/4, so rounding
// it to the nearest integer gives a.  Then S mod q = sum_j y_j ((M/m_j) mod q) - a (M mod q) mod q.
HFE_HD float crt_frac_add(float frac, uint32_t y, float rcp) { return fmaf((float)y, rcp, frac); }
HFE_HD uint64_t crt_round(float frac) { return (uint64_t)(frac + 0.5f); }
// acc = sum_j y_j ((M/m_j) mod q) (any value below 2^64), a from crt_round.
HFE_HD uint64_t crt_finish(uint64_t acc, uint64_t a, uint64_t M_mod_q, const Mod& md) {
  return sub_mod(barrett64(acc, md.q, md.mu), barrett64(a * M_mod_q, md.q, md.mu), md.q);
}

}  // namespace hfe
