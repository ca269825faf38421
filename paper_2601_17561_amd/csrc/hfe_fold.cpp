// Normalise and fold (Algorithm 2, Section 4.3, Appendix C.2): keys, the encryption of inner-product
// score numerators, the fold of blocks of score ciphertexts and the decryption of its result (kernels in
// k_fold.hip).
//
// A block of rho ciphertexts ct_c (slot j of ct_c: the inner product of query column c with database
// entry j, at scale 2^20, level 4) becomes ceil(rho / k) ciphertexts
//   ct'_r = RS_{q_1}( Rot_{r k}( sum_{r' < min(k, rho - r k)} Rot_{r'}( f( RS_{q_4}(ct_{r k + r'} * Ecd(1 / count_{r k + r'})) ) ) ) )
// at level 0, scale 2^24: the normalisation into scores (a plaintext product and RS by the 36-bit q_4),
// the folding polynomial f of degree 7 in the three levels of q_3 .. q_1 (near 2^23; five products
// with relinearisation, constants encoded at the scales that make the terms they join equal; the last
// product is not rescaled), the rotations of Section 4.3 (slot i of Rot_r(v) holds v_(i - r)) and the
// sum over the k ciphertexts of a group at level 1, where the key-switching error is far below the
// scale, and one rescale per group.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hfe_internal.h"
#include "hfe_slots.h"

namespace hfe {
namespace {

using u128 = unsigned __int128;
uint64_t mm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

hfe_status hip_err(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? HFE_ENOMEM : HFE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define FD_LAUNCH(expr)                              \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_err(_e, #expr); \
  } while (0)

hfe_status put(DevBuf& b, const void* host, size_t bytes, hipStream_t s) {
  HFE_TRY(b.alloc(bytes, s));
  FD_LAUNCH(hipMemcpyAsync(b.ptr, host, bytes, hipMemcpyHostToDevice, s));
  FD_LAUNCH(hipStreamSynchronize(s));
  return HFE_OK;
}

template <class T>
T* handle_of(const void* h, uint32_t kind) {
  if (!h) return nullptr;
  const HandleBase* b = static_cast<const HandleBase*>(h);
  return b->kind == kind ? static_cast<T*>(const_cast<void*>(h)) : nullptr;
}

// The `count` largest primes below 2^bits that are 1 mod 2^17, descending.
void ntt_primes_below(int bits, int count, uint64_t* out) {
  const uint64_t step = 1ull << 17;
  uint64_t q = ((1ull << bits) - 1) / step * step + 1;
  if (q >= (1ull << bits)) q -= step;
  for (int got = 0; got < count; q -= step)
    if (is_prime_u64(q)) out[got++] = q;
}

// f(x) = sum_j c_j x^j, the folding polynomial of Appendix C.2 (degree 7, k = 16).
constexpr double kCoeffs[8] = {0.004105, -0.173510, -2.528271, 24.347349, 124.161550, -412.746212, 376.961251,
                               106.553952};
constexpr int kLogIn = 20, kLogMu = 40, kLogF = 24, kWBits = 30;
constexpr int kRotLevel = 1;  // level of the rotations and group sums

// The scales of x, x^2, x^4 and of the terms of f, and the integer constants k_0 .. k_7 of f: each scale
// is one product and one quotient of doubles, in a fixed order, so that every implementation of the
// schedule reaches the same constants.
void fold_schedule(const uint64_t* q, double* sched, int64_t* k) {
#pragma clang fp contract(off)
  const double q1 = (double)q[1], q2 = (double)q[2], q3 = (double)q[3], q4 = (double)q[4];
  const double S1 = (double)(1ull << (kLogIn + kLogMu)) / q4;  // x = RS_{q_4}(ct mu), level 3
  const double S2 = (S1 * S1) / q3;                            // x^2, level 2
  const double S4 = (S2 * S2) / q2;                            // x^4, level 1
  const double F = (double)(1ull << kLogF);                    // the folded result, level 0
  const double G = F * q1;                                     // f at level 1 (exact: 24 + 23 bits)
  const double U = G / S4;                                     // x^4 (c4 + c5 x + x^2 L3) has scale G
  const double T3 = (U * q2) / S2;                             // x^2 L3 has scale U
  const double T1 = (G * q2) / S2;                             // x^2 L1 has scale G
  const double E7 = (T3 * q3) / S1, E3 = (T1 * q3) / S1, E5 = (U * q3) / S1, E1 = (G * q3) / S1;
  const double c0 = kCoeffs[0] * G, c1 = kCoeffs[1] * E1, c2 = kCoeffs[2] * T1, c3 = kCoeffs[3] * E3;
  const double c4 = kCoeffs[4] * U, c5 = kCoeffs[5] * E5, c6 = kCoeffs[6] * T3, c7 = kCoeffs[7] * E7;
  k[0] = round_half_up(c0);
  k[1] = round_half_up(c1);
  k[2] = round_half_up(c2);
  k[3] = round_half_up(c3);
  k[4] = round_half_up(c4);
  k[5] = round_half_up(c5);
  k[6] = round_half_up(c6);
  k[7] = round_half_up(c7);
  const double v[8] = {S1, S2, S4, F, U, T3, T1, G};
  std::memcpy(sched, v, sizeof(v));
}

// 5^e mod 2N for the exponent of Rot_r: X -> X^(5^-r), 5^-r = 5^(N/2 - r) mod 2N.
uint32_t rot_galois(int logn, int r) {
  const uint64_t n = 1ull << logn, half = n / 2;
  return (uint32_t)pow_mod(5, (half - (uint64_t)r % half) % half, 2 * n);
}

uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Rotations a fold of blocks of rho uses: 1 .. min(k, rho) - 1, then r k for 1 <= r < ceil(rho / k).
std::vector<int32_t> rot_amounts(int k, int rho) {
  std::vector<int32_t> a;
  for (int r = 1; r < std::min(k, rho); ++r) a.push_back(r);
  for (int r = 1; r < (rho + k - 1) / k; ++r) a.push_back(r * k);
  return a;
}

uint64_t residue(int64_t v, uint64_t q) {
  const int64_t r = v % (int64_t)q;
  return (uint64_t)(r < 0 ? r + (int64_t)q : r);
}

SlotMap slots_upto(int l, bool with_p) {
  SlotMap m{};
  for (int i = 0; i <= l; ++i) m.z[i] = (int8_t)i;
  if (with_p) m.z[l + 1] = 5;
  return m;
}

// NTT of a small signed polynomial at every slot: [6][N] residues.
hfe_status small_hat(const hfe_foldkeys* F, const std::vector<int64_t>& poly, DevBuf& out, hipStream_t s) {
  const int n = 1 << F->C.logn;
  std::vector<uint64_t> h((size_t)kFoldSlots * n);
  for (int z = 0; z < kFoldSlots; ++z)
    for (int t = 0; t < n; ++t) h[(size_t)z * n + t] = residue(poly[(size_t)t], F->C.mod[z].q);
  HFE_TRY(put(out, h.data(), h.size() * 8, s));
  for (int z = 0; z < kFoldSlots; ++z)
    FD_LAUNCH(launch_ntt_fwd(out.as<uint64_t>() + (size_t)z * n, 1, n, F->C.tab[z], false, s));
  return HFE_OK;
}

// One key-switching key from s_from to s at level l (slots 0 .. l and p, digits 0 .. l), written as
// doubles [s][i][2][N] to dst; kappa numbers its random columns.
hfe_status make_ks_key(const hfe_foldkeys* F, uint64_t seed, int kappa, int l, const DevBuf& from_hat, double* dst,
                       hipStream_t s) {
  const int n = 1 << F->C.logn;
  const int nsl = l + 2;
  const SlotMap zm = slots_upto(l, true);
  DevBuf coef;
  HFE_TRY(coef.alloc((size_t)nsl * (l + 1) * 2 * n * 8, s));
  FD_LAUNCH(launch_fold_key_coeffs(F->C, seed, kappa, l, zm, F->cdt.as<uint64_t>(), coef.as<uint64_t>(), s));
  for (int sp = 0; sp < nsl; ++sp)
    FD_LAUNCH(launch_ntt_fwd(coef.as<uint64_t>() + (size_t)sp * (l + 1) * 2 * n, (int64_t)(l + 1) * 2, n,
                             F->C.tab[zm.z[sp]], false, s));
  KeyGadget gk{};
  const uint64_t p = F->C.mod[5].q;
  for (int sp = 0; sp < nsl; ++sp) {
    const uint64_t zq = F->C.mod[zm.z[sp]].q;
    for (int i = 0; i <= l; ++i) {
      uint64_t g = p % zq;  // p (Q_l / q_i) mod z
      for (int j = 0; j <= l; ++j)
        if (j != i) g = mm(g, F->C.mod[j].q % zq, zq);
      gk.v[sp][i] = (double)g;
    }
  }
  FD_LAUNCH(launch_fold_key_finish(F->C, l, zm, coef.as<uint64_t>(), F->s_hat.as<uint64_t>(), from_hat.as<uint64_t>(),
                                   gk, dst, s));
  FD_LAUNCH(hipStreamSynchronize(s));
  return HFE_OK;
}

hfe_status fold_keygen_impl(int logn, int k, int rho, uint64_t seed, hfe_foldkeys* F) {
  hipStream_t s = nullptr;
  F->kind = kFoldKeys;
  F->stream = s;
  F->k = k;
  F->rho = rho;
  FoldConsts& C = F->C;
  std::memset(&C, 0, sizeof(C));
  C.logn = logn;
  const int n = 1 << logn;
  uint64_t big[3], small[3];
  ntt_primes_below(36, 3, big);    // q_0, p, q_4
  ntt_primes_below(23, 3, small);  // q_1 .. q_3
  const uint64_t primes[kFoldSlots] = {big[0], small[0], small[1], small[2], big[2], big[1]};
  std::vector<uint64_t> tab;
  for (int z = 0; z < kFoldSlots; ++z) {
    const uint64_t q = primes[z];
    C.zd[z] = (double)q;
    C.zinv[z] = 1.0 / (double)q;
    C.mod[z] = make_mod(q);
    C.pid[z] = z < 5 ? (uint32_t)z : 16u;
    ntt_tables_host(q, logn, tab);  // psi | psi_sh | ipsi | ipsi_sh
    std::vector<double> td(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      td[(size_t)i] = (double)tab[(size_t)i];
      td[(size_t)n + i] = (double)tab[2 * (size_t)n + i];
    }
    NttTabOwner& o = F->tabs[z];
    HFE_TRY(put(o.buf, td.data(), td.size() * sizeof(double), s));
    o.tab.psi_d = o.buf.as<double>();
    o.tab.ipsi_d = o.buf.as<double>() + n;
    o.tab.q = q;
    o.tab.qd = (double)q;
    o.tab.qinv = 1.0 / (double)q;
    o.tab.n_inv_d = (double)inv_mod((uint64_t)n % q, q);
    o.tab.logn = logn;
    C.tab[z] = o.tab;
  }
  int64_t kc[8];
  fold_schedule(primes, F->sched, kc);
  for (int j = 0; j < 8; ++j) F->ksum[j] = (uint64_t)kc[j];

  // the secret: the 32 coefficients whose words (stream FSec, sub 0) are smallest, ties by index,
  // sign from the parity of the word at the same position of sub 1
  {
    std::vector<std::pair<uint64_t, int>> w((size_t)n);
    for (int t = 0; t < n; ++t) {
      const Philox4 b = philox4x64_10(seed, stream_tag(kFSec, 0), (uint64_t)t >> 2, 0, 0, 0);
      w[(size_t)t] = {b.v[t & 3], t};
    }
    std::sort(w.begin(), w.end());
    F->s_host.assign((size_t)n, 0);
    for (int h = 0; h < kFoldH && h < n; ++h) {
      const int t = w[(size_t)h].second;
      const Philox4 u = philox4x64_10(seed, stream_tag(kFSec, 1), (uint64_t)t >> 2, 0, 0, 0);
      F->s_host[(size_t)t] = (u.v[t & 3] & 1) ? -1 : 1;
    }
  }
  std::vector<int64_t> sv((size_t)n);
  for (int t = 0; t < n; ++t) sv[(size_t)t] = F->s_host[(size_t)t];
  HFE_TRY(small_hat(F, sv, F->s_hat, s));
  {
    uint64_t cdt[19];
    if (cdt_table_quad_impl(cdt) != 0) return fail(HFE_EDEVICE, "Gaussian table");
    HFE_TRY(put(F->cdt, cdt, sizeof(cdt), s));
  }

  // relinearisation keys at levels 1 .. 3 (s^2 -> s)
  {
    std::vector<int64_t> s2((size_t)n, 0);
    for (int i = 0; i < n; ++i)
      if (sv[(size_t)i])
        for (int j = 0; j < n; ++j)
          if (sv[(size_t)j]) {
            const int64_t v = sv[(size_t)i] * sv[(size_t)j];
            const int t = i + j;
            if (t < n)
              s2[(size_t)t] += v;
            else
              s2[(size_t)(t - n)] -= v;
          }
    DevBuf s2_hat;
    HFE_TRY(small_hat(F, s2, s2_hat, s));
    int64_t off = 0;
    for (int l = 1; l <= 3; ++l) {
      F->relin_off[l] = off;
      off += (int64_t)(l + 2) * (l + 1) * 2 * n;
    }
    HFE_TRY(F->relin.alloc((size_t)off * sizeof(double), s));
    for (int l = 1; l <= 3; ++l)
      HFE_TRY(make_ks_key(F, seed, l - 1, l, s2_hat, F->relin.as<double>() + F->relin_off[l], s));
  }
  // rotation keys at level 1 (s(X^g) -> s) and the NTT-point permutations of the automorphisms
  F->amounts = rot_amounts(k, rho);
  const size_t na = F->amounts.size();
  const size_t per_key = (size_t)(kRotLevel + 2) * (kRotLevel + 1) * 2 * n;
  HFE_TRY(F->rot.alloc(std::max<size_t>(1, na) * per_key * sizeof(double), s));
  std::vector<int32_t> perm(std::max<size_t>(1, na) * n, 0);
  for (size_t a = 0; a < na; ++a) {
    const uint32_t g = rot_galois(logn, F->amounts[a]);
    std::vector<int64_t> sg((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
      const uint64_t t = (uint64_t)i * g % (2ull * n);
      if (t >= (uint64_t)n)
        sg[(size_t)(t - n)] = -sv[(size_t)i];
      else
        sg[(size_t)t] = sv[(size_t)i];
    }
    DevBuf sg_hat;
    HFE_TRY(small_hat(F, sg, sg_hat, s));
    HFE_TRY(make_ks_key(F, seed, 3 + (int)a, kRotLevel, sg_hat, F->rot.as<double>() + a * per_key, s));
    // output point i is a(psi^(e_i g)) with e_i = 2 brv(i) + 1: the input point k with e_k = e_i g mod 2N
    for (int i = 0; i < n; ++i) {
      const uint64_t e = (2ull * brv((uint32_t)i, logn) + 1) * g % (2ull * n);
      perm[a * n + (size_t)i] = (int32_t)brv((uint32_t)((e - 1) / 2), logn);
    }
  }
  HFE_TRY(put(F->perm, perm.data(), perm.size() * sizeof(int32_t), s));

  // the slot transforms' tables
  {
    const int m = n / 2;
    std::vector<double> W(m), Z(2 * (size_t)m);
    std::vector<int32_t> pos(m), kj(m);
    slot_tables(logn, W.data(), Z.data(), pos.data(), kj.data());
    HFE_TRY(put(F->slot_w, W.data(), W.size() * 8, s));
    HFE_TRY(put(F->slot_z, Z.data(), Z.size() * 8, s));
    HFE_TRY(put(F->slot_pos, pos.data(), pos.size() * 4, s));
    HFE_TRY(put(F->slot_k, kj.data(), kj.size() * 4, s));
  }
  FD_LAUNCH(hipStreamSynchronize(s));
  return HFE_OK;
}

// ------------------------------------------------------------------ evaluator steps on arrays of n items
struct Ev {
  const hfe_foldkeys* F;
  const FoldConsts& C;
  hipStream_t s;
  int64_t n;   // items
  int64_t N;   // ring degree
};

int64_t ct_words(const Ev& e, int l) { return e.n * 2 * (l + 1) * e.N; }

SlotFactor const_res(const FoldConsts& C, int64_t k, int nsl) {
  SlotFactor r{};
  for (int j = 0; j < nsl; ++j) r.v[j] = (double)residue(k, C.mod[j].q);
  return r;
}

// RS by q_l: x [n][2][l+1][N] -> out [n][2][l][N]; with pm ([n][l+1][N], NTT domain), RS by q_l of the
// plaintext product x pm, the product formed as the two passes load x.
hfe_status rescale(const Ev& e, const uint64_t* x, int l, uint64_t* out, const uint64_t* pm = nullptr) {
  DevBuf cen;
  HFE_TRY(cen.alloc((size_t)e.n * 2 * e.N * 8, e.s));
  FoldInv ia;
  ia.src = x + l * e.N;
  ia.si = (l + 1) * e.N;
  ia.zm.z[0] = (int8_t)l;
  ia.nsl = 1;
  ia.mode = 1;
  ia.dst = cen.ptr;
  ia.di = e.N;
  ia.pm = pm;
  ia.pmi = (l + 1) * e.N;
  FD_LAUNCH(launch_fold_inv(e.C, ia, e.n * 2, e.s));
  FoldLift la;
  la.cen = cen.as<int64_t>();
  la.pm = pm;
  la.pmi = (l + 1) * e.N;
  la.x = x;
  la.xi = 2 * (l + 1) * e.N;
  la.xp = (l + 1) * e.N;
  la.out = out;
  la.oi = 2 * l * e.N;
  la.op = l * e.N;
  la.zm = slots_upto(l - 1, false);
  la.nsl = l;
  const uint64_t ql = e.C.mod[l].q;
  for (int j = 0; j < l; ++j) la.inv.v[j] = (double)inv_mod(ql % e.C.mod[j].q, e.C.mod[j].q);
  FD_LAUNCH(launch_fold_lift(e.C, la, e.n, e.s));
  return HFE_OK;
}

// The sums of a key switch at level l: digits of the polynomial src (item stride si, slots 0 .. l at stride
// N), or of the product src y (the a parts of a tensor) when y is given; acc [n][2][l+1][N] the sums at
// q_0 .. q_l (NTT domain), accp [n][2][N] the sums at p, centered (coefficients).  keys + kidx[item] * kstride
// is the item's key.
hfe_status ks_sums(const Ev& e, int l, const uint64_t* src, const uint64_t* y, int64_t si, const double* keys,
                   int64_t kstride, const int32_t* kidx, DevBuf& acc, DevBuf& accp) {
  DevBuf dig;
  HFE_TRY(dig.alloc((size_t)e.n * (l + 1) * e.N * 8, e.s));
  HFE_TRY(acc.alloc((size_t)e.n * 2 * (l + 1) * e.N * 8, e.s));
  HFE_TRY(accp.alloc((size_t)e.n * 2 * e.N * 8, e.s));
  FoldInv ia;
  ia.src = src;
  ia.y = y;
  ia.si = si;
  ia.ss = e.N;
  ia.dst = dig.ptr;
  ia.di = (l + 1) * e.N;
  ia.ds = e.N;
  ia.zm = slots_upto(l, false);
  ia.nsl = l + 1;
  ia.mode = 2;
  for (int i = 0; i <= l; ++i) {
    const uint64_t qi = e.C.mod[i].q;
    uint64_t qhat = 1;  // (Q_l / q_i) mod q_i
    for (int j = 0; j <= l; ++j)
      if (j != i) qhat = mm(qhat, e.C.mod[j].q % qi, qi);
    ia.f.v[i] = (double)inv_mod(qhat, qi);
  }
  FD_LAUNCH(launch_fold_inv(e.C, ia, e.n, e.s));
  FD_LAUNCH(launch_fold_ks_mac(e.C, l, ia, dig.as<uint64_t>(), keys, kstride, kidx, acc.as<uint64_t>(),
                               accp.as<int64_t>(), e.n, e.s));
  return HFE_OK;
}

// Key switch at level l (see ks_sums): RS_p of the sums plus the addends that `tail` names, to tail.out.
hfe_status key_switch(const Ev& e, int l, const uint64_t* src, const uint64_t* y, int64_t si, const double* keys,
                      int64_t kstride, const int32_t* kidx, FoldLift tail) {
  DevBuf acc, accp;
  HFE_TRY(ks_sums(e, l, src, y, si, keys, kstride, kidx, acc, accp));
  tail.cen = accp.as<int64_t>();
  tail.x = acc.as<uint64_t>();
  tail.xi = 2 * (l + 1) * e.N;
  tail.xp = (l + 1) * e.N;
  tail.zm = slots_upto(l, false);
  tail.nsl = l + 1;
  const uint64_t p = e.C.mod[5].q;
  for (int j = 0; j <= l; ++j) tail.inv.v[j] = (double)inv_mod(p % e.C.mod[j].q, e.C.mod[j].q);
  FD_LAUNCH(launch_fold_lift(e.C, tail, e.n, e.s));
  return HFE_OK;
}

// x y with relinearisation at level l (the tensor's d2 formed in the digit pass, d0 and d1 in the last
// pass).  Rescaled (the default): p (d0, d1) plus the key switch's sums divided by p q_l in one rounding,
// out [n][2][l][N], plus add2 (level l - 1); otherwise the relinearised product (d0, d1) + RS_p(sums),
// [n][2][l + 1][N], plus add2 (level l).
hfe_status mul(const Ev& e, const uint64_t* x, const uint64_t* y, int l, uint64_t* out, bool rescaled = true,
               const uint64_t* add2 = nullptr) {
  const int64_t per = (l + 1) * e.N;
  const double* key = e.F->relin.as<double>() + e.F->relin_off[l];
  FoldLift tail;
  tail.tx = x;
  tail.ty = y;
  tail.ti = 2 * per;
  tail.tp = per;
  tail.out = out;
  if (!rescaled) {
    tail.oi = 2 * per;
    tail.op = per;
    if (add2) {
      tail.add2 = add2;
      tail.a2i = 2 * per;
      tail.a2p = per;
    }
    return key_switch(e, l, x + per, y + per, 2 * per, key, 0, nullptr, tail);
  }
  DevBuf acc, accp, cen;
  HFE_TRY(ks_sums(e, l, x + per, y + per, 2 * per, key, 0, nullptr, acc, accp));
  HFE_TRY(cen.alloc((size_t)e.n * 2 * e.N * 8, e.s));
  FD_LAUNCH(launch_fold_relin_center(e.C, l, acc.as<uint64_t>(), accp.as<int64_t>(), x, y, e.n, cen.as<int64_t>(),
                                     e.s));
  const int64_t po = l * e.N;  // the output's slots q_0 .. q_{l-1}
  tail.cen = cen.as<int64_t>();
  tail.x = acc.as<uint64_t>();
  tail.xi = 2 * per;
  tail.xp = per;
  tail.oi = 2 * po;
  tail.op = po;
  if (add2) {
    tail.add2 = add2;
    tail.a2i = 2 * po;
    tail.a2p = po;
  }
  tail.zm = slots_upto(l - 1, false);
  tail.nsl = l;
  tail.has_tscale = 1;
  const uint64_t p = e.C.mod[5].q, ql = e.C.mod[l].q;
  for (int j = 0; j < l; ++j) {
    const uint64_t qj = e.C.mod[j].q;
    tail.inv.v[j] = (double)inv_mod(mm(p % qj, ql % qj, qj), qj);  // (p q_l)^-1
    tail.tscale.v[j] = (double)inv_mod(ql % qj, qj);               // p (d0, d1) (p q_l)^-1 = (d0, d1) q_l^-1
  }
  FD_LAUNCH(launch_fold_lift(e.C, tail, e.n, e.s));
  return HFE_OK;
}

// RS(k x) at level l -> level l - 1, kept at the slots of level `to` (a mod-drop), then + c.  u: the
// residues of x's last slot in coefficients, [n][2][N] (shared by the constants: the transform of k x_l is
// k times that of x_l).
hfe_status const_term(const Ev& e, const uint64_t* x, const uint64_t* u, int l, int64_t k, int to, int64_t c,
                      DevBuf& out) {
  HFE_TRY(out.alloc((size_t)ct_words(e, to) * 8, e.s));
  FoldLift la;
  la.ures = u;
  la.cl = l;
  la.ku = (double)residue(k, e.C.mod[l].q);
  la.x = x;
  la.xi = 2 * (l + 1) * e.N;
  la.xp = (l + 1) * e.N;
  la.has_xmul = 1;
  la.xmul = const_res(e.C, k, to + 1);
  la.cres = const_res(e.C, c, to + 1);
  la.out = out.as<uint64_t>();
  la.oi = 2 * (to + 1) * e.N;
  la.op = (to + 1) * e.N;
  la.zm = slots_upto(to, false);
  la.nsl = to + 1;
  const uint64_t ql = e.C.mod[l].q;
  for (int j = 0; j <= to; ++j) la.inv.v[j] = (double)inv_mod(ql % e.C.mod[j].q, e.C.mod[j].q);
  FD_LAUNCH(launch_fold_lift(e.C, la, e.n, e.s));
  return HFE_OK;
}

// Rotations at level 1 of the items src[u] of x ([.][2][2][N]) by the amounts with key index amt[u]
// (device arrays of m entries): out [m][2][2][N].
hfe_status rotate(const hfe_foldkeys* F, hipStream_t s, const uint64_t* x, const int32_t* src, const int32_t* amt,
                  int64_t m, uint64_t* out) {
  if (m == 0) return HFE_OK;
  const int64_t N = 1ll << F->C.logn;
  const int l = kRotLevel, nsl = kRotLevel + 1;
  const int64_t per = 2 * nsl * N;
  Ev e{F, F->C, s, m, N};
  DevBuf P;
  HFE_TRY(P.alloc((size_t)m * per * 8, s));
  FD_LAUNCH(launch_fold_perm(F->C, x, src, amt, F->perm.as<int32_t>(), P.as<uint64_t>(), m, nsl, s));
  FoldLift tail;
  tail.add = P.as<uint64_t>();  // sigma(b), to part 0 only
  tail.ai = per;
  tail.ap = 0;
  tail.out = out;
  tail.oi = per;
  tail.op = nsl * N;
  return key_switch(e, l, P.as<uint64_t>() + nsl * N, nullptr, per, F->rot.as<double>(),
                    (int64_t)(l + 2) * (l + 1) * 2 * N, amt, tail);
}

hfe_status fold_impl(const hfe_foldkeys* F, const hfe_fct* in, const int32_t* counts, int64_t rho, hipStream_t s,
                     hfe_fct* out, hipEvent_t* ev) {
  const FoldConsts& C = F->C;
  const int64_t n = in->count, N = 1ll << C.logn;
  const int logn = C.logn;
  Ev e{F, C, s, n, N};
  const int64_t* k = reinterpret_cast<const int64_t*>(F->ksum);
  if (ev) FD_LAUNCH(hipEventRecord(ev[0], s));

  // mu = Ecd(1 / counts) at scale 2^40, NTT at q_0 .. q_4
  DevBuf flag, w, m, mu;
  HFE_TRY(flag.alloc(sizeof(uint32_t), s));
  FD_LAUNCH(hipMemsetAsync(flag.ptr, 0, sizeof(uint32_t), s));
  HFE_TRY(w.alloc((size_t)n * (N / 2) * 8, s));
  FD_LAUNCH(launch_fold_weights(counts, n * (N / 2), 1, w.as<int64_t>(), flag.as<uint32_t>(), s));
  HFE_TRY(m.alloc((size_t)n * N * 8, s));
  FD_LAUNCH(launch_fold_encode(w.as<int64_t>(), n, logn, std::ldexp(1.0, kLogMu - kWBits), F->slot_w.as<double>(),
                               F->slot_z.as<double>(), F->slot_pos.as<int32_t>(), m.as<int64_t>(), s));
  w.reset();
  HFE_TRY(mu.alloc((size_t)n * 5 * N * 8, s));
  FD_LAUNCH(launch_fold_fwd(C, m.as<int64_t>(), N, 0, mu.as<uint64_t>(), 5 * N, N, slots_upto(4, false), 5, n, s));
  m.reset();
  if (ev) FD_LAUNCH(hipEventRecord(ev[1], s));

  // x = RS_{q_4}(ct mu), level 3 (the product formed where the rescale loads it)
  DevBuf x3;
  HFE_TRY(x3.alloc((size_t)ct_words(e, 3) * 8, s));
  HFE_TRY(rescale(e, in->ct.as<uint64_t>(), 4, x3.as<uint64_t>(), mu.as<uint64_t>()));
  mu.reset();
  if (ev) FD_LAUNCH(hipEventRecord(ev[2], s));

  // f(x) = (c0 + c1 x) + x^2 (c2 + c3 x) + x^4 ((c4 + c5 x) + x^2 (c6 + c7 x)) at level 1, scale G: the
  // sums formed in the last passes of the products (inner = x^2 L3 + L2; t1 = x^2 L1 + L0; f = x^4 inner + t1)
  DevBuf x2, x4, L0, L1, L2, L3, inner, t1, f;
  HFE_TRY(x2.alloc((size_t)ct_words(e, 2) * 8, s));
  HFE_TRY(mul(e, x3.as<uint64_t>(), x3.as<uint64_t>(), 3, x2.as<uint64_t>()));
  {
    DevBuf u3;  // x's slot q_3 in coefficients, for the four constant terms
    HFE_TRY(u3.alloc((size_t)n * 2 * N * 8, s));
    FoldInv ia;
    ia.src = x3.as<uint64_t>() + 3 * N;
    ia.si = 4 * N;
    ia.zm.z[0] = 3;
    ia.nsl = 1;
    ia.dst = u3.ptr;
    ia.di = N;
    FD_LAUNCH(launch_fold_inv(C, ia, n * 2, s));
    HFE_TRY(const_term(e, x3.as<uint64_t>(), u3.as<uint64_t>(), 3, k[7], 2, k[6], L3));
    HFE_TRY(const_term(e, x3.as<uint64_t>(), u3.as<uint64_t>(), 3, k[3], 2, k[2], L1));
    HFE_TRY(const_term(e, x3.as<uint64_t>(), u3.as<uint64_t>(), 3, k[5], 1, k[4], L2));
    HFE_TRY(const_term(e, x3.as<uint64_t>(), u3.as<uint64_t>(), 3, k[1], 1, k[0], L0));
  }
  x3.reset();
  HFE_TRY(x4.alloc((size_t)ct_words(e, 1) * 8, s));
  HFE_TRY(mul(e, x2.as<uint64_t>(), x2.as<uint64_t>(), 2, x4.as<uint64_t>()));
  HFE_TRY(inner.alloc((size_t)ct_words(e, 1) * 8, s));
  HFE_TRY(mul(e, x2.as<uint64_t>(), L3.as<uint64_t>(), 2, inner.as<uint64_t>(), true, L2.as<uint64_t>()));
  HFE_TRY(t1.alloc((size_t)ct_words(e, 1) * 8, s));
  HFE_TRY(mul(e, x2.as<uint64_t>(), L1.as<uint64_t>(), 2, t1.as<uint64_t>(), true, L0.as<uint64_t>()));
  x2.reset();
  HFE_TRY(f.alloc((size_t)ct_words(e, 1) * 8, s));
  HFE_TRY(mul(e, x4.as<uint64_t>(), inner.as<uint64_t>(), 1, f.as<uint64_t>(), false, t1.as<uint64_t>()));
  if (ev) FD_LAUNCH(hipEventRecord(ev[3], s));

  // rotations inside each group, the group sums, and the rotation of group r by r k
  const int kf = F->k;
  const int64_t blocks = n / rho, gpb = (rho + kf - 1) / kf, groups = blocks * gpb;
  auto amount_index = [&](int a) -> int32_t {
    for (size_t i = 0; i < F->amounts.size(); ++i)
      if (F->amounts[i] == a) return (int32_t)i;
    return -1;
  };
  std::vector<int32_t> src1, amt1, beg(1, 0), mem, src2, amt2;
  for (int64_t b = 0; b < blocks; ++b)
    for (int64_t r = 0; r < gpb; ++r) {
      const int64_t first = b * rho + r * kf;
      mem.push_back((int32_t)(first * 2));
      for (int64_t rp = 1; rp < std::min<int64_t>(kf, rho - r * kf); ++rp) {
        mem.push_back((int32_t)(src1.size() * 2 + 1));
        src1.push_back((int32_t)(first + rp));
        amt1.push_back(amount_index((int)rp));
      }
      beg.push_back((int32_t)mem.size());
      if (r) {
        src2.push_back((int32_t)(b * gpb + r));
        amt2.push_back(amount_index((int)(r * kf)));
      }
    }
  for (int32_t a : amt1)
    if (a < 0) return fail(HFE_EINVAL, "rotation amount without a key");
  for (int32_t a : amt2)
    if (a < 0) return fail(HFE_EINVAL, "rotation amount without a key");
  DevBuf d_src1, d_amt1, d_beg, d_mem, d_src2, d_amt2, R1, R2;
  auto up = [&](DevBuf& b, const std::vector<int32_t>& v) -> hfe_status {
    if (v.empty()) return HFE_OK;
    return put(b, v.data(), v.size() * 4, s);
  };
  HFE_TRY(up(d_src1, src1));
  HFE_TRY(up(d_amt1, amt1));
  HFE_TRY(up(d_beg, beg));
  HFE_TRY(up(d_mem, mem));
  HFE_TRY(up(d_src2, src2));
  HFE_TRY(up(d_amt2, amt2));
  const int nr = kRotLevel + 1;
  const int64_t per = 2 * nr * N;
  if (!src1.empty()) {
    HFE_TRY(R1.alloc(src1.size() * per * 8, s));
    HFE_TRY(rotate(F, s, f.as<uint64_t>(), d_src1.as<int32_t>(), d_amt1.as<int32_t>(), (int64_t)src1.size(),
                   R1.as<uint64_t>()));
  }
  DevBuf sums;
  HFE_TRY(sums.alloc((size_t)groups * per * 8, s));
  FD_LAUNCH(launch_fold_group_sum(C, f.as<uint64_t>(), R1.as<uint64_t>(), d_beg.as<int32_t>(), d_mem.as<int32_t>(),
                                  sums.as<uint64_t>(), groups, nr, s));
  if (!src2.empty()) {
    HFE_TRY(R2.alloc(src2.size() * per * 8, s));
    HFE_TRY(rotate(F, s, sums.as<uint64_t>(), d_src2.as<int32_t>(), d_amt2.as<int32_t>(), (int64_t)src2.size(),
                   R2.as<uint64_t>()));
    FD_LAUNCH(launch_fold_scatter(C, R2.as<uint64_t>(), d_src2.as<int32_t>(), sums.as<uint64_t>(),
                                  (int64_t)src2.size(), nr, s));
  }
  // RS by q_1: the folded sums at level 0, scale F
  HFE_TRY(out->ct.alloc((size_t)groups * 2 * N * 8, s));
  {
    Ev eg{F, C, s, groups, N};
    HFE_TRY(rescale(eg, sums.as<uint64_t>(), kRotLevel, out->ct.as<uint64_t>()));
  }
  if (ev) FD_LAUNCH(hipEventRecord(ev[4], s));
  out->count = groups;
  out->level = 0;
  out->scale = F->sched[3];
  uint32_t bad = 0;
  FD_LAUNCH(hipMemcpyAsync(&bad, flag.ptr, sizeof(bad), hipMemcpyDeviceToHost, s));
  FD_LAUNCH(hipStreamSynchronize(s));
  if (bad) return fail(HFE_EINVAL, "counts must lie in 1 .. 2^24");
  return HFE_OK;
}

}  // namespace
}  // namespace hfe

using namespace hfe;

extern "C" {

hfe_status hfe_fold_keygen(uint32_t log_n, uint32_t k, uint32_t rho, uint64_t seed, hfe_foldkeys** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  if (log_n < 6 || log_n > (uint32_t)kMaxLogN) return fail(HFE_EINVAL, "the fold needs 6 <= log_n <= 14");
  if (k < 1 || k > (1u << (log_n - 1))) return fail(HFE_EINVAL, "k must lie in 1 .. N/2");
  if (rho < 1 || rho > (1u << (log_n - 1))) return fail(HFE_EINVAL, "rho must lie in 1 .. N/2");
  hfe_foldkeys* F = new (std::nothrow) hfe_foldkeys();
  if (!F) return fail(HFE_ENOMEM, "host allocation failed");
  hfe_status st = fold_keygen_impl((int)log_n, (int)k, (int)rho, seed, F);
  if (st != HFE_OK) {
    delete F;
    return st;
  }
  *out = F;
  return HFE_OK;
}

hfe_status hfe_fold_encrypt(const hfe_foldkeys* fk, const int32_t* ip, int64_t count, uint64_t seed, void* stream,
                            hfe_fct** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_foldkeys* F = handle_of<hfe_foldkeys>(fk, kFoldKeys);
  if (!F || !ip) return fail(HFE_EINVAL, "invalid fold keys or ip");
  if (count < 1 || count > (1 << 20)) return fail(HFE_ESHAPE, "count must be 1 .. 2^20");
  const FoldConsts& C = F->C;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = 1ll << C.logn;
  hfe_fct* X = new (std::nothrow) hfe_fct();
  if (!X) return fail(HFE_ENOMEM, "host allocation failed");
  X->kind = kFct;
  X->stream = s;
  X->keys = F;
  X->level = kFoldLevels;
  X->count = count;
  X->scale = (double)(1 << kLogIn);
  auto run = [&]() -> hfe_status {
    DevBuf flag, w, m;
    HFE_TRY(flag.alloc(sizeof(uint32_t), s));
    FD_LAUNCH(hipMemsetAsync(flag.ptr, 0, sizeof(uint32_t), s));
    HFE_TRY(w.alloc((size_t)count * (N / 2) * 8, s));
    FD_LAUNCH(launch_fold_weights(ip, count * (N / 2), 0, w.as<int64_t>(), flag.as<uint32_t>(), s));
    HFE_TRY(m.alloc((size_t)count * N * 8, s));
    FD_LAUNCH(launch_fold_encode(w.as<int64_t>(), count, C.logn, std::ldexp(1.0, kLogIn), F->slot_w.as<double>(),
                                 F->slot_z.as<double>(), F->slot_pos.as<int32_t>(), m.as<int64_t>(), s));
    FD_LAUNCH(launch_fold_add_errors(C, seed, F->cdt.as<uint64_t>(), m.as<int64_t>(), count, s));
    HFE_TRY(X->ct.alloc((size_t)count * 2 * 5 * N * 8, s));
    FD_LAUNCH(launch_fold_fwd(C, m.as<int64_t>(), N, 0, X->ct.as<uint64_t>(), 2 * 5 * N, N, slots_upto(4, false), 5,
                              count, s));
    FD_LAUNCH(launch_fold_encrypt(C, seed, F->s_hat.as<uint64_t>(), X->ct.as<uint64_t>(), count, s));
    uint32_t bad = 0;
    FD_LAUNCH(hipMemcpyAsync(&bad, flag.ptr, sizeof(bad), hipMemcpyDeviceToHost, s));
    FD_LAUNCH(hipStreamSynchronize(s));
    if (bad) return fail(HFE_EINVAL, "inner products must lie in -2^24 .. 2^24");
    return HFE_OK;
  };
  hfe_status st = run();
  if (st != HFE_OK) {
    delete X;
    return st;
  }
  *out = X;
  return HFE_OK;
}

hfe_status hfe_fold(const hfe_foldkeys* fk, const hfe_fct* in, const int32_t* counts, int64_t rho, void* stream,
                    hfe_fct** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_foldkeys* F = handle_of<hfe_foldkeys>(fk, kFoldKeys);
  const hfe_fct* X = handle_of<hfe_fct>(in, kFct);
  if (!F || !X || !counts) return fail(HFE_EINVAL, "invalid fold keys, ciphertexts or counts");
  if (X->keys != F) return fail(HFE_EINVAL, "the ciphertexts were made under other fold keys");
  if (X->level != kFoldLevels) return fail(HFE_ELEVEL, "the fold takes ciphertexts at level 4 (fresh encryptions)");
  if (rho < 1 || rho > F->rho) return fail(HFE_ESHAPE, "rho must lie in 1 .. the rho of the keys");
  if (X->count % rho) return fail(HFE_ESHAPE, "the count must be a multiple of rho");
  hipStream_t s = (hipStream_t)stream;
  hfe_fct* O = new (std::nothrow) hfe_fct();
  if (!O) return fail(HFE_ENOMEM, "host allocation failed");
  O->kind = kFct;
  O->stream = s;
  O->keys = F;
  hfe_status st = HFE_OK;
  hipEvent_t* ev = nullptr;
  if (profiling()) {
    for (auto& e : O->ev)
      if (st == HFE_OK && hipEventCreate(&e) != hipSuccess) st = fail(HFE_EDEVICE, "hipEventCreate");
    ev = O->ev;
  }
  if (st == HFE_OK) st = fold_impl(F, X, counts, rho, s, O, ev);
  if (st != HFE_OK) {
    delete O;
    return st;
  }
  *out = O;
  return HFE_OK;
}

hfe_status hfe_fold_decrypt(const hfe_foldkeys* fk, const hfe_fct* ct, double* values, void* stream) {
  const hfe_foldkeys* F = handle_of<hfe_foldkeys>(fk, kFoldKeys);
  const hfe_fct* X = handle_of<hfe_fct>(ct, kFct);
  if (!F || !X || !values) return fail(HFE_EINVAL, "invalid fold keys, ciphertexts or values");
  if (X->keys != F) return fail(HFE_EINVAL, "the ciphertexts were made under other fold keys");
  if (X->level != 0) return fail(HFE_ELEVEL, "decryption takes folded ciphertexts (level 0)");
  hipStream_t s = (hipStream_t)stream;
  const FoldConsts& C = F->C;
  const int64_t N = 1ll << C.logn;
  DevBuf h, m;
  HFE_TRY(h.alloc((size_t)X->count * N * 8, s));
  HFE_TRY(m.alloc((size_t)X->count * N * 8, s));
  FD_LAUNCH(launch_fold_dec_products(C, X->ct.as<uint64_t>(), F->s_hat.as<uint64_t>(), h.as<uint64_t>(), X->count, s));
  FoldInv ia;
  ia.src = h.as<uint64_t>();
  ia.si = N;
  ia.dst = m.ptr;
  ia.di = N;
  ia.nsl = 1;
  ia.mode = 1;
  FD_LAUNCH(launch_fold_inv(C, ia, X->count, s));
  FD_LAUNCH(launch_fold_decode(m.as<int64_t>(), X->count, C.logn, F->slot_w.as<double>(), F->slot_z.as<double>(),
                               F->slot_k.as<int32_t>(), 1.0 / X->scale, values, s));
  FD_LAUNCH(hipStreamSynchronize(s));
  return HFE_OK;
}

hfe_status hfe_fold_profile_ms(const hfe_fct* ct, float* ms, int32_t n) {
  const hfe_fct* X = handle_of<hfe_fct>(ct, kFct);
  if (!X || !ms || n < 0 || n > 4) return fail(HFE_EINVAL, "invalid ciphertexts, ms or n (0 .. 4)");
  if (!X->ev[0]) return fail(HFE_EINVAL, "the ciphertexts were not made by a profiled fold");
  FD_LAUNCH(hipEventSynchronize(X->ev[4]));
  for (int i = 0; i < n; ++i) FD_LAUNCH(hipEventElapsedTime(&ms[i], X->ev[i], X->ev[i + 1]));
  return HFE_OK;
}

}  // extern "C"

namespace hfe {
// Coefficient-form residues of a fold ciphertext array, [count][2][level + 1][N], for hfe_export.
hfe_status fold_export(const hfe_fct* X, DevBuf& out, hipStream_t s) {
  const FoldConsts& C = X->keys->C;
  const int64_t N = 1ll << C.logn;
  const int l = X->level;
  HFE_TRY(out.alloc((size_t)X->count * 2 * (l + 1) * N * 8, s));
  FoldInv ia;
  ia.src = X->ct.as<uint64_t>();
  ia.si = (l + 1) * N;
  ia.ss = N;
  ia.dst = out.ptr;
  ia.di = (l + 1) * N;
  ia.ds = N;
  ia.zm = slots_upto(l, false);
  ia.nsl = l + 1;
  FD_LAUNCH(launch_fold_inv(C, ia, X->count * 2, s));
  FD_LAUNCH(hipStreamSynchronize(s));
  return HFE_OK;
}
}  // namespace hfe
