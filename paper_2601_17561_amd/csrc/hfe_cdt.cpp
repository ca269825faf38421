// Cumulative table of the discrete Gaussian error distribution, computed in quad precision.
//
// rho(x) = exp(-x^2 / (2 sigma^2)) with sigma = 3.2 (so x^2 / (2 sigma^2) = 25 x^2 / 512 is
// exact in binary), restricted to |x| <= 19.  T[j] = floor(2^64 * P(|e| <= j)) for j < 19, with
// P(|e| <= j) = (rho(0) + 2 sum_{x=1..j} rho(x)) / (rho(0) + 2 sum_{x=1..19} rho(x)).
// The 113-bit significand leaves about 2^-46 of absolute error on 2^64 P, far below the
// distance of these values to an integer.  Built with g++ (libquadmath); no HIP headers.
#include <quadmath.h>
#include <stdint.h>

namespace hfe {

int cdt_table_quad_impl(uint64_t* dst) {
  __float128 rho[20];
  for (int x = 0; x <= 19; ++x) rho[x] = expq(-(__float128)(25 * x * x) / (__float128)512);
  __float128 z = rho[0];
  for (int x = 1; x <= 19; ++x) z += 2 * rho[x];
  __float128 cum = rho[0];
  const __float128 two64 = ldexpq((__float128)1, 64);
  for (int j = 0; j < 19; ++j) {
    if (j) cum += 2 * rho[j];
    __float128 v = floorq(cum / z * two64);
    if (v < 0 || v >= two64) return -1;
    dst[j] = (uint64_t)v;
  }
  return 0;
}

}  // namespace hfe
