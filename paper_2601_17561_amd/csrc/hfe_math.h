// Integer arithmetic shared by host and device code of the library: Philox4x64-10,
// 64-bit high products, modular reduction (Barrett, Shoup) for primes below 2^36.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HFE_HD __host__ __device__ __forceinline__

namespace hfe {

// High 64 bits of a 64 x 64 product.
HFE_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// Philox4x64 with 10 rounds (Salmon et al., SC 2011): multipliers and Weyl key increments
// from the published definition.
struct Philox4 {
  uint64_t v[4];
};

HFE_HD Philox4 philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                             uint64_t c3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0 = mulhi64(M0, x0), lo0 = M0 * x0;
    uint64_t hi1 = mulhi64(M1, x2), lo1 = M1 * x2;
    uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
  Philox4 o;
  o.v[0] = x0;
  o.v[1] = x1;
  o.v[2] = x2;
  o.v[3] = x3;
  return o;
}

// Stream purposes of the random draws (key1 = purpose << 32 | sub).
enum : uint64_t { kQSec = 1, kDbSec = 2, kDbA = 3, kDbE = 4, kQA = 5, kQE = 6 };
constexpr uint32_t kPrimeIdP = 16;  // stream id of the special prime
HFE_HD uint64_t stream_tag(uint64_t purpose, uint64_t sub) { return (purpose << 32) | sub; }

// Per-prime reduction constants.
struct Mod {
  uint64_t q;
  uint64_t mu;     // floor(2^64 / q)
  uint64_t bound;  // floor(2^64 / q) * q: largest multiple of q below 2^64 (rejection bound)
};

HFE_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}
HFE_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

// x mod q for any 64-bit x (Barrett with mu = floor(2^64/q); at most two corrections).
HFE_HD uint64_t barrett64(uint64_t x, uint64_t q, uint64_t mu) {
  uint64_t r = x - mulhi64(x, mu) * q;
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  return r;
}

// Shoup multiplication a * w mod q with w_sh = floor(w * 2^64 / q), w < q, any a < 2^64.
HFE_HD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t w_sh, uint64_t q) {
  uint64_t h = mulhi64(a, w_sh);
  uint64_t r = a * w - h * q;
  return r >= q ? r - q : r;
}

// Shoup quotient floor(w * 2^64 / q) for w < q < 2^63, by binary long division.
HFE_HD uint64_t shoup_quot(uint64_t w, uint64_t q) {
  uint64_t r = w, quo = 0;
  for (int i = 63; i >= 0; --i) {
    r <<= 1;
    if (r >= q) {
      r -= q;
      quo |= 1ull << i;
    }
  }
  return quo;
}

// a * b mod q for a, b < q < 2^36 (no precomputation): split b at 28 bits so every
// partial product fits 64 bits.
HFE_HD uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t q, uint64_t mu) {
  uint64_t b0 = b & ((1ull << 28) - 1), b1 = b >> 28;
  uint64_t r0 = barrett64(a * b0, q, mu);
  uint64_t r1 = barrett64(a * b1, q, mu);
  r1 = barrett64(r1 << 28, q, mu);
  return add_mod(r0, r1, q);
}

// Signed integer (|x| < 2^63) to its residue mod q.
HFE_HD uint64_t from_signed(int64_t x, uint64_t q, uint64_t mu) {
  if (x >= 0) return barrett64((uint64_t)x, q, mu);
  uint64_t r = barrett64((uint64_t)(-x), q, mu);
  return r ? q - r : 0;
}

// Residue in [0, q) to its centered representative in (-q/2, q/2) (q odd).
HFE_HD int64_t centered(uint64_t r, uint64_t q) {
  return r > (q >> 1) ? (int64_t)r - (int64_t)q : (int64_t)r;
}

// Uniform residue mod q at element (i0, i1) of a stream: word (i0 & 3) of block
// (i0 >> 2, i1, 0, 0); on rejection the first accepted word of blocks (i0, i1, attempt, 0).
HFE_HD uint64_t uniform_at(uint64_t seed, uint64_t key1, uint64_t i0, uint64_t i1,
                           const Mod& m) {
  Philox4 b = philox4x64_10(seed, key1, i0 >> 2, i1, 0, 0);
  uint64_t w = b.v[i0 & 3];
  if (w < m.bound) return barrett64(w, m.q, m.mu);
  // Each attempt fails with probability < 2^-112 for a 36-bit q; the cap only bounds the loop.
  for (uint64_t attempt = 1; attempt <= 64; ++attempt) {
    Philox4 y = philox4x64_10(seed, key1, i0, i1, attempt, 0);
    for (int j = 0; j < 4; ++j)
      if (y.v[j] < m.bound) return barrett64(y.v[j], m.q, m.mu);
  }
  return 0;
}

// The CDT sample of one word pair: magnitude = #{j : w >= T[j]}, negative iff magnitude > 0 and the
// sign word is odd.
HFE_HD int32_t cdt_sample(uint64_t w, uint64_t sw, const uint64_t* cdt) {
  int32_t mag = 0;
#pragma unroll
  for (int j = 0; j < 19; ++j) mag += (w >= cdt[j]) ? 1 : 0;
  return ((sw & 1) && mag) ? -mag : mag;
}

// Discrete Gaussian at element (i0, i1): block (i0 >> 1, i1, 0, 0), words (2h, 2h + 1) with
// h = i0 & 1; magnitude = #{j : w >= T[j]}, negative iff magnitude > 0 and the sign word is odd.
HFE_HD int32_t gaussian_at(uint64_t seed, uint64_t key1, uint64_t i0, uint64_t i1,
                           const uint64_t* cdt) {
  Philox4 b = philox4x64_10(seed, key1, i0 >> 1, i1, 0, 0);
  const bool h = (i0 & 1) != 0;  // words 2h, 2h + 1 of the block (selected, not indexed: registers)
  return cdt_sample(h ? b.v[2] : b.v[0], h ? b.v[3] : b.v[1], cdt);
}

// The Gaussians of elements (2u, i1) and (2u + 1, i1) from their one block: the same values as two
// gaussian_at calls for half the Philox evaluations.
HFE_HD void gaussian_pair_at(uint64_t seed, uint64_t key1, uint64_t u, uint64_t i1, const uint64_t* cdt,
                             int32_t& e0, int32_t& e1) {
  Philox4 b = philox4x64_10(seed, key1, u, i1, 0, 0);
  e0 = cdt_sample(b.v[0], b.v[1], cdt);
  e1 = cdt_sample(b.v[2], b.v[3], cdt);
}

}  // namespace hfe
