// Host build of the library's exact-arithmetic helpers (paper_2601_17561_amd/csrc/hfe_exact.h), for
// the CPU tests: each function applies one helper, as the kernels call it, to arrays of operands
// given by the test, which compares the results with exact integer arithmetic in Python.
// The exhaustive sweeps compare with C's integer remainder in the same loop.
#include <stdint.h>

#include "../../paper_2601_17561_amd/csrc/hfe_exact.h"
#include "../../paper_2601_17561_amd/csrc/hfe_slots.h"

using namespace hfe;

static constexpr RnsModConsts kRns = make_rns_mod_consts();
static constexpr P2BaseConsts kP2 = make_p2_base_consts();

extern "C" {

// The fold's slot encoder (hfe_slots.h) on w (N/2 integers) at scale 2^e: out = N integer coefficients.
void xc_slot_encode(const int64_t* w, int logn, int e, int64_t* out) {
  const int64_t n = int64_t(1) << logn, m = n / 2;
  double* W = new double[m];
  double* Z = new double[2 * m];
  int32_t* pos = new int32_t[m];
  int32_t* kj = new int32_t[m];
  double* z = new double[m];
  double* scratch = new double[2 * m];
  slot_tables(logn, W, Z, pos, kj);
  for (int64_t j = 0; j < m; ++j) z[j] = (double)w[j] * ldexp(1.0, e);
  slot_encode_host(z, logn, W, Z, pos, scratch, out);
  delete[] W;
  delete[] Z;
  delete[] pos;
  delete[] kj;
  delete[] z;
  delete[] scratch;
}

// out[i] = a[i] w[i] mod q by the fp64 product of the transforms (qinv = RN(1/q) as the tables hold it).
void xc_mulmod_d(const uint64_t* a, const uint64_t* w, int64_t n, uint64_t q, uint64_t* out) {
  const double qd = (double)q, qinv = 1.0 / qd;
  for (int64_t i = 0; i < n; ++i) out[i] = (uint64_t)mulmod_d((double)a[i], (double)w[i], qd, qinv);
}

// out[i] = the centered product of a[i] (|a| <= 16q) and w[i] (in [0, q)), as int64.
void xc_mulmod_c_d(const int64_t* a, const uint64_t* w, int64_t n, uint64_t q, int64_t* out) {
  const double qd = (double)q, qinv = 1.0 / qd;
  for (int64_t i = 0; i < n; ++i) out[i] = (int64_t)mulmod_c_d((double)a[i], (double)w[i], qd, qinv);
}

// out[i] = reduce_c_d(x[i]) then residue_of_c, as uint64.
void xc_reduce_c_d(const int64_t* x, int64_t n, uint64_t q, uint64_t* out) {
  const double qd = (double)q, qinv = 1.0 / qd;
  for (int64_t i = 0; i < n; ++i) out[i] = (uint64_t)residue_of_c(reduce_c_d((double)x[i], qd, qinv), qd);
}

// A forward transform of length 2^logn through ct_butterfly_c (the stage order of the kernels, twiddles
// w[m + j] as in the tables, w given as integers), then reduce_c_d: out[i] in [0, q).  Also returns the
// largest magnitude met between stages.
int64_t xc_ntt_signed(const int64_t* in, const uint64_t* w, int logn, uint64_t q, uint64_t* out) {
  const int n = 1 << logn;
  const double qd = (double)q, qinv = 1.0 / qd;
  double* a = new double[n];
  for (int i = 0; i < n; ++i) a[i] = (double)in[i];
  double big = 0.0;
  for (int m = 1, t = n / 2; m < n; m *= 2, t /= 2)
    for (int j = 0; j < m; ++j)
      for (int i = 2 * j * t; i < 2 * j * t + t; ++i) {
        ct_butterfly_c(a[i], a[i + t], (double)w[m + j], qd, qinv);
        big = __builtin_fabs(a[i]) > big ? __builtin_fabs(a[i]) : big;
        big = __builtin_fabs(a[i + t]) > big ? __builtin_fabs(a[i + t]) : big;
      }
  for (int i = 0; i < n; ++i) out[i] = (uint64_t)residue_of_c(reduce_c_d(a[i], qd, qinv), qd);
  delete[] a;
  return (int64_t)big;
}

// Mismatches of mod_u32 against x % m: every x < 2^24, every x within 3 of a multiple of m up to 2^32,
// 2^32 - 1, and n_random pseudo-random x (splitmix64).
int64_t xc_mod_u32_sweep(uint32_t m, int64_t n_random) {
  const uint32_t magic = magic_u32(m);
  int64_t bad = 0;
  for (uint32_t x = 0; x < (1u << 24); ++x) bad += mod_u32(x, m, magic) != x % m;
  for (uint64_t k = 1; k * m < (1ull << 32) + 4; ++k)
    for (int d = -3; d <= 3; ++d) {
      const int64_t x = (int64_t)(k * m) + d;
      if (x >= 0 && x < (int64_t)(1ull << 32)) bad += mod_u32((uint32_t)x, m, magic) != (uint32_t)x % m;
    }
  bad += mod_u32(0xFFFFFFFFu, m, magic) != 0xFFFFFFFFu % m;
  uint64_t z = 0x9E3779B97F4A7C15ull * m;
  for (int64_t i = 0; i < n_random; ++i) {
    z += 0x9E3779B97F4A7C15ull;
    uint64_t t = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    t = (t ^ (t >> 27)) * 0x94D049BB133111EBull;
    const uint32_t x = (uint32_t)(t ^ (t >> 31));
    bad += mod_u32(x, m, magic) != x % m;
  }
  return bad;
}

// The inverse transform of the kernels on signed values (rounds of up to three Gentleman-Sande stages,
// each round starting from centered representatives, the last one scaling by n_inv), twiddles iw[m + j]
// as in the tables: out[i] in [0, q).  Returns the largest magnitude met inside a round.
int64_t xc_intt_signed(const int64_t* in, const uint64_t* iw, int logn, uint64_t q, uint64_t n_inv, uint64_t* out) {
  const int n = 1 << logn;
  const double qd = (double)q, qinv = 1.0 / qd;
  double* a = new double[n];
  for (int i = 0; i < n; ++i) a[i] = (double)in[i];
  double big = 0.0;
  int t = 1, left = logn;
  while (left > 0) {
    const int S = left >= 3 ? 3 : left;
    const bool last = left == S;
    const int G = 1 << S;
    for (int g = 0; g < (n >> S); ++g) {
      const int B = g / t, r = g - B * t, base = B * G * t + r;
      double x[8];
      for (int k = 0; k < G; ++k) x[k] = reduce_c_d(a[base + k * t], qd, qinv);
      for (int s = 0; s < S; ++s) {
        const int h = 1 << s, m = n / (2 * h * t);
        for (int k = 0; k < G; ++k) {
          if (k & h) continue;
          const int w = m + (B << (S - 1 - s)) + (k >> (s + 1));
          const double U = x[k], V = x[k + h];
          const double d = U - V;
          big = __builtin_fabs(d) > big ? __builtin_fabs(d) : big;
          x[k] = U + V;
          x[k + h] = mulmod_c_d(d, (double)iw[w], qd, qinv);
          big = __builtin_fabs(x[k]) > big ? __builtin_fabs(x[k]) : big;
        }
      }
      if (last)
        for (int k = 0; k < G; ++k) x[k] = residue_of_c(mulmod_c_d(x[k], (double)n_inv, qd, qinv), qd);
      for (int k = 0; k < G; ++k) a[base + k * t] = x[k];
    }
    t <<= S;
    left -= S;
  }
  for (int i = 0; i < n; ++i) out[i] = (uint64_t)a[i];
  delete[] a;
  return (int64_t)big;
}

void xc_mod_small(const uint32_t* x, int64_t n, uint32_t m, uint32_t* out) {
  const uint32_t magic = (uint32_t)(((1ull << 32) + m - 1) / m);
  for (int64_t i = 0; i < n; ++i) out[i] = mod_small(x[i], m, magic);
}

// Mismatches of mod_small against x % m over every x < limit.
int64_t xc_mod_small_sweep(uint32_t m, uint32_t limit) {
  const uint32_t magic = (uint32_t)(((1ull << 32) + m - 1) / m);
  int64_t bad = 0;
  for (uint32_t x = 0; x < limit; ++x) bad += mod_small(x, m, magic) != x % m;
  return bad;
}

void xc_mod_f64(const int64_t* x, int64_t n, int64_t m, int64_t* out) {
  const double rcp = 1.0 / (double)m;
  for (int64_t i = 0; i < n; ++i) out[i] = mod_f64(x[i], m, rcp);
}

// balanced residue modulo kRnsMods[j], with the constants the kernels use
void xc_balanced_mod(const int64_t* x, int64_t n, int j, int32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = balanced_mod_by(x[i], kRns.m[j], kRns.magic[j], kRns.t24[j]);
}

// n^2-form digits for base kP2Bases[j]
void xc_p2_digits(const int64_t* x, int64_t n, int j, int32_t* M, int32_t* Mp) {
  for (int64_t i = 0; i < n; ++i) p2_digits_by(x[i], kP2.n[j], kP2.m[j], kP2.magic_n[j], kP2.rcp_m[j], M[i], Mp[i]);
}

// The same two n^2 helpers for any base n, with the constants the n^2 modulus chain passes its
// kernels (ceil(2^32 / n), RN(1 / n), RN(1 / n^2)).
void xc_p2_digits_n(const int64_t* x, int64_t cnt, int32_t n, int32_t* M, int32_t* Mp) {
  const uint32_t magic = (uint32_t)(((1ull << 32) + (uint64_t)n - 1) / (uint64_t)n);
  const int32_t m = n * n;
  const double rcp_m = 1.0 / (double)m;
  for (int64_t i = 0; i < cnt; ++i) p2_digits_by(x[i], n, m, magic, rcp_m, M[i], Mp[i]);
}
void xc_p2_acc_mod_n(const int32_t* g0, const int32_t* g1, int64_t cnt, int32_t n, uint32_t* out) {
  const int32_t m = n * n;
  for (int64_t i = 0; i < cnt; ++i) out[i] = p2_acc_mod(g0[i], g1[i], n, m, 1.0 / (double)n, 1.0 / (double)m);
}

// RNS epilogue: int32 sums -> residue modulo kRnsMods[j]
void xc_rns_acc_mod(const int32_t* s, int64_t n, int j, uint32_t* out) {
  const RnsAccConsts c = rns_acc_consts(kRns.m[j], kRns.magic[j]);
  for (int64_t i = 0; i < n; ++i) out[i] = rns_acc_mod(s[i], kRns.m[j], kRns.magic[j], c);
}

// Mismatches of the RNS epilogue against the exact remainder, over every int32 sum s = lo + k step.
int64_t xc_rns_acc_mod_sweep(int j, int64_t lo, int64_t step, int64_t count) {
  const uint32_t m = kRns.m[j];
  const RnsAccConsts c = rns_acc_consts(m, kRns.magic[j]);
  int64_t bad = 0;
  for (int64_t k = 0; k < count; ++k) {
    const int64_t s = lo + k * step;
    const int64_t want = ((s % (int64_t)m) + m) % m;
    bad += (int64_t)rns_acc_mod((int32_t)s, m, kRns.magic[j], c) != want;
  }
  return bad;
}

// n^2 epilogue: (G0, G1) -> (G0 + n G1) mod n^2 for base kP2Bases[j]
void xc_p2_acc_mod(const int32_t* g0, const int32_t* g1, int64_t n, int j, uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = p2_acc_mod(g0[i], g1[i], kP2.n[j], kP2.m[j], kP2.rcp_n[j], kP2.rcp_m[j]);
}

// CRT of one entry per column of s ([nm][cnt] residues s_j = S mod m_j), as the kernels take it:
// y_j = s_j inv_j mod m_j (RNS: multiply-high quotient; n^2: the fp64 quotient), the fp32 fraction
// sum, a = its rounding, out = S mod q.  Also returns a for the test.
void xc_crt(const uint32_t* s, int64_t cnt, int nm, const uint32_t* m, const uint32_t* inv, const float* rcp,
            const uint64_t* Mj_mod_q, uint64_t M_mod_q, uint64_t q, uint64_t mu, int p2, uint64_t* out,
            uint64_t* a_out) {
  Mod md;
  md.q = q;
  md.mu = mu;
  md.bound = 0;
  for (int64_t e = 0; e < cnt; ++e) {
    float frac = 0.f;
    uint64_t acc = 0;
    for (int j = 0; j < nm; ++j) {
      const uint32_t x = s[(int64_t)j * cnt + e];
      uint32_t y;
      if (p2) {
        y = (uint32_t)mod_f64((int64_t)x * inv[j], m[j], 1.0 / (double)m[j]);
      } else {
        const uint32_t magic = (uint32_t)(((1ull << 32) + m[j] - 1) / m[j]);
        y = mod_small(x * inv[j], m[j], magic);
      }
      frac = crt_frac_add(frac, y, rcp[j]);
      acc += (uint64_t)y * Mj_mod_q[j];
    }
    const uint64_t a = crt_round(frac);
    a_out[e] = a;
    out[e] = crt_finish(acc, a, M_mod_q, md);
  }
}

}  // extern "C"
