// Host-side number theory of the library: primality, modular inverses, primitive roots and
// the negacyclic NTT twiddle tables (Longa-Naehrig bit-reversed ordering).
#include <vector>

#include "hfe_internal.h"

namespace hfe {

namespace {
using u128 = unsigned __int128;

uint64_t mulmod_u128(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

bool miller_rabin_witness(uint64_t n, uint64_t a, uint64_t d, int s) {
  uint64_t x = 1, base = a % n, e = d;
  while (e) {
    if (e & 1) x = mulmod_u128(x, base, n);
    base = mulmod_u128(base, base, n);
    e >>= 1;
  }
  if (x == 1 || x == n - 1) return false;
  for (int r = 1; r < s; ++r) {
    x = mulmod_u128(x, x, n);
    if (x == n - 1) return false;
  }
  return true;  // a witnesses compositeness
}

uint32_t bit_reverse(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}
}  // namespace

// Deterministic Miller-Rabin for 64-bit n (bases: the first 12 primes).
bool is_prime_u64(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : bases) {
    if (n % b == 0) return n == b;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : bases)
    if (miller_rabin_witness(n, a, d, s)) return false;
  return true;
}

uint64_t pow_mod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, b = a % q;
  while (e) {
    if (e & 1) r = mulmod_u128(r, b, q);
    b = mulmod_u128(b, b, q);
    e >>= 1;
  }
  return r;
}

// a^-1 mod q for gcd(a, q) = 1, any modulus q (prime or not: the n^2 chain's moduli are squares), by
// the extended Euclidean algorithm; 0 when no inverse exists.
uint64_t inv_mod(uint64_t a, uint64_t q) {
  int64_t t0 = 0, t1 = 1;
  uint64_t r0 = q, r1 = a % q;
  while (r1) {
    const uint64_t k = r0 / r1;
    const uint64_t r2 = r0 - k * r1;
    const int64_t t2 = t0 - (int64_t)k * t1;  // |t| <= q < 2^63
    r0 = r1;
    r1 = r2;
    t0 = t1;
    t1 = t2;
  }
  if (r0 != 1) return 0;
  return t0 < 0 ? (uint64_t)(t0 + (int64_t)q) : (uint64_t)t0;
}

Mod make_mod(uint64_t q) {
  Mod m;
  m.q = q;
  m.mu = (uint64_t)(((u128)1 << 64) / q);
  m.bound = m.mu * q;
  return m;
}

uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

uint64_t primitive_2n_root(uint64_t q, int logn) {
  // prime factors of q - 1
  std::vector<uint64_t> f;
  uint64_t m = q - 1;
  for (uint64_t d = 2; d * d <= m; ++d) {
    if (m % d == 0) {
      f.push_back(d);
      while (m % d == 0) m /= d;
    }
  }
  if (m > 1) f.push_back(m);
  uint64_t g = 2;
  for (;; ++g) {
    bool gen = true;
    for (uint64_t p : f)
      if (pow_mod(g, (q - 1) / p, q) == 1) {
        gen = false;
        break;
      }
    if (gen) break;
  }
  return pow_mod(g, (q - 1) >> (logn + 1), q);
}

void ntt_tables_host(uint64_t q, int logn, std::vector<uint64_t>& out) {
  const uint32_t n = 1u << logn;
  const uint64_t psi = primitive_2n_root(q, logn);
  const uint64_t ipsi = inv_mod(psi, q);
  std::vector<uint64_t> pw(n), ipw(n);
  pw[0] = ipw[0] = 1;
  for (uint32_t i = 1; i < n; ++i) {
    pw[i] = mulmod_u128(pw[i - 1], psi, q);
    ipw[i] = mulmod_u128(ipw[i - 1], ipsi, q);
  }
  out.assign(4 * (size_t)n, 0);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t b = bit_reverse(i, logn);
    out[i] = pw[b];
    out[n + i] = shoup(pw[b], q);
    out[2 * n + i] = ipw[b];
    out[3 * n + i] = shoup(ipw[b], q);
  }
}

}  // namespace hfe
