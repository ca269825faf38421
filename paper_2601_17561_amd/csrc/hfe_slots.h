// The slot encoding of CKKS at ring degree N (the canonical embedding), for the normalisation of the
// fold: N/2 slots, slot j the evaluation at zeta^(g_j), zeta = e^(i pi / N), g_j = 5^j mod 2N.
//
// The g_j are exactly the residues 1 mod 4 below 2N (5 generates them), g_j = 1 + 4 k_j, and
// zeta^(g_j M) = i for M = N/2.  With u_i = m_i + i m_(i+M) (i < M) a real polynomial m satisfies
//   m(zeta^(g_j)) = sum_{i<M} u_i zeta^i w^(i k_j),   w = zeta^4 = e^(2 pi i / M),
// a DFT of length M of the twisted u_i zeta^i.  So the encoder is a length-M inverse DFT of the slots
// placed at k_j, an untwist by zeta^-i / M and a rounding of the real and imaginary parts.
//
// The inverse DFT is the iterative radix-2 decimation-in-time transform on bit-reversed input
// (natural-order output), twiddles W[u] = e^(-2 pi i u / M); each butterfly and the untwist are fixed
// sequences of IEEE fp64 products and sums without fused multiply-adds, so that any implementation that
// performs the same operations on the same tables (cos and sin of the C library) reaches the same
// rounded coefficients.  The functions are host and device code: the kernel calls them, and a host build
// is compared with an independent implementation by the CPU tests.
#pragma once

#include <math.h>
#include <stdint.h>

#include "hfe_math.h"

namespace hfe {

// (a, c) -> (a + w c, a - w c) for complex a, c, w (w c = (wr cr - wi ci, wr ci + wi cr)).
HFE_HD void slot_butterfly(double& ar, double& ai, double& cr, double& ci, double wr, double wi) {
#pragma clang fp contract(off)
  const double pr = wr * cr - wi * ci;
  const double pi = wr * ci + wi * cr;
  const double xr = ar, xi = ai;
  ar = xr + pr;
  ai = xi + pi;
  cr = xr - pr;
  ci = xi - pi;
}

// u = (x conj(zeta^i)) / M with zeta^i = (c, s): ((xr c + xi s) inv_m, (xi c - xr s) inv_m).
HFE_HD void slot_untwist(double xr, double xi, double c, double s, double inv_m, double& ur, double& ui) {
#pragma clang fp contract(off)
  const double tr = xr * c + xi * s;
  const double ti = xi * c - xr * s;
  ur = tr * inv_m;
  ui = ti * inv_m;
}

// x = u zeta^i with zeta^i = (c, s): (ur c - ui s, ur s + ui c) (the decoder's twist).
HFE_HD void slot_twist(double ur, double ui, double c, double s, double& xr, double& xi) {
#pragma clang fp contract(off)
  xr = ur * c - ui * s;
  xi = ur * s + ui * c;
}

HFE_HD int64_t round_half_up(double v) {
#pragma clang fp contract(off)
  return (int64_t)floor(v + 0.5);
}

HFE_HD uint32_t slot_brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Tables for ring degree 2^logn, M = N/2 (host): W[2u], W[2u+1] = cos, -sin of 2 pi u / M (u < M/2);
// Z[2i], Z[2i+1] = cos, sin of pi i / N (i < M); pos[j] = brv(k_j) (where slot j enters the transform),
// kj[j] = k_j = (g_j - 1) / 4 (where the decoder's transform leaves slot j).
inline void slot_tables(int logn, double* W, double* Z, int32_t* pos, int32_t* kj) {
  const int64_t n = int64_t(1) << logn, m = n / 2;
  const int lm = logn - 1;
  for (int64_t u = 0; u < m / 2; ++u) {
    const double a = 2.0 * M_PI * (double)u / (double)m;
    W[2 * u] = cos(a);
    W[2 * u + 1] = -sin(a);
  }
  for (int64_t i = 0; i < m; ++i) {
    const double a = M_PI * (double)i / (double)n;
    Z[2 * i] = cos(a);
    Z[2 * i + 1] = sin(a);
  }
  uint64_t g = 1;
  for (int64_t j = 0; j < m; ++j) {
    const uint32_t k = (uint32_t)((g - 1) / 4);
    kj[j] = (int32_t)k;
    pos[j] = (int32_t)slot_brv(k, lm);
    g = g * 5 % (uint64_t)(2 * n);
  }
}

// Host encoder with the kernel's operations (the reference the CPU tests compare): real slot values
// z[j] (exact doubles) -> integer coefficients m[0 .. N).
inline void slot_encode_host(const double* z, int logn, const double* W, const double* Z, const int32_t* pos,
                             double* scratch, int64_t* m) {
  const int64_t n = int64_t(1) << logn, M = n / 2;
  double* xr = scratch;
  double* xi = scratch + M;
  for (int64_t j = 0; j < M; ++j) {
    xr[pos[j]] = z[j];
    xi[pos[j]] = 0.0;
  }
  for (int64_t half = 1; half < M; half *= 2) {
    const int64_t step = M / (2 * half);
    for (int64_t b = 0; b < M / 2; ++b) {
      const int64_t grp = b / half, t = b - grp * half;
      const int64_t ia = grp * 2 * half + t, ic = ia + half;
      slot_butterfly(xr[ia], xi[ia], xr[ic], xi[ic], W[2 * t * step], W[2 * t * step + 1]);
    }
  }
  const double inv_m = 1.0 / (double)M;
  for (int64_t i = 0; i < M; ++i) {
    double ur, ui;
    slot_untwist(xr[i], xi[i], Z[2 * i], Z[2 * i + 1], inv_m, ur, ui);
    m[i] = round_half_up(ur);
    m[M + i] = round_half_up(ui);
  }
}

}  // namespace hfe
