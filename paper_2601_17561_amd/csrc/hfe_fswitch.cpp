// FormatSwitch (Appendix C.1): key generation, the client's transmission encryption and the switch
// of transmission ciphertexts in R_{N_T} to the CCMM's query ciphertext (kernels in k_fswitch.hip).
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hfe_internal.h"

namespace hfe {
namespace {

using u128 = unsigned __int128;
uint64_t mm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

hfe_status hip_err(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? HFE_ENOMEM : HFE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define FS_LAUNCH(expr)                              \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_err(_e, #expr); \
  } while (0)

hfe_status put(DevBuf& b, const void* host, size_t bytes) {
  HFE_TRY(b.alloc(bytes, nullptr));
  FS_LAUNCH(hipMemcpy(b.ptr, host, bytes, hipMemcpyHostToDevice));
  return HFE_OK;
}

uint64_t residue(int v, uint64_t q) { return v >= 0 ? (uint64_t)v : q - (uint64_t)(-v); }

// Slot z of a switch at level l: q_z for z <= l, p (the keys' prime index L) for z = l + 1.
int key_index(const hfe_keys* K, int l, int z) { return z <= l ? z : K->L; }

hfe_status fs_consts(const hfe_keys* K, int l, int log_n_t, FsConsts& C) {
  std::memset(&C, 0, sizeof(C));
  C.level = l;
  C.nz = l + 2;
  C.k = K->k;
  C.logn_q = (int)K->P.log_n_q;
  C.logn_t = log_n_t;
  C.rho = 1 << (log_n_t - C.logn_q);
  C.d2 = K->P.d2;
  uint64_t lo = ~0ull, hi = 0;
  for (int z = 0; z < C.nz; ++z) {
    const int x = key_index(K, l, z);
    const uint64_t q = K->primes[x];
    C.zd[z] = (double)q;
    C.zinv[z] = 1.0 / (double)q;
    C.mod[z] = K->mods[x];
    C.pid[z] = K->prime_id[x];
    C.tab[z] = K->tab_q[x].tab;
    lo = q < lo ? q : lo;
    hi = q > hi ? q : hi;
  }
  // digits below q_i enter the signed transforms of every slot modulus z as they are (below 2z, the
  // transforms' input bound), and every rescale corrects once each way: both need the moduli within a
  // factor 2 of each other
  if (hi >= 2 * lo) return fail(HFE_EINVAL, "FormatSwitch needs q_0 .. q_level and p within a factor 2");
  const uint64_t p = K->primes[K->L];
  const uint64_t ql = K->primes[l];
  const int dl = delta_log(K, l);
  for (int i = 0; i <= l; ++i) {
    const uint64_t qi = K->primes[i];
    uint64_t qhat = 1;  // (Q' / q_i) mod q_i
    for (int j = 0; j <= l; ++j)
      if (j != i) qhat = mm(qhat, K->primes[j] % qi, qi);
    C.ghat[i] = (double)inv_mod(qhat, qi);
    C.pinv[i] = (double)inv_mod(p % qi, qi);
    C.qlinv[i] = i < l ? (double)inv_mod(ql % qi, qi) : 0.0;
    C.scale[i] = (double)mm(pow_mod(2, (uint64_t)dl, qi), ql % qi, qi);
    for (int z = 0; z < C.nz; ++z) {
      const uint64_t zq = K->primes[key_index(K, l, z)];
      uint64_t g = p % zq;  // p (Q' / q_i) mod z
      for (int j = 0; j <= l; ++j)
        if (j != i) g = mm(g, K->primes[j] % zq, zq);
      C.gk[z][i] = g;
    }
  }
  return HFE_OK;
}

hfe_status fs_keygen_impl(const hfe_keys* K, int l, int log_n_t, uint64_t seed, hfe_fskeys* F) {
  F->kind = kFsKeys;
  F->stream = nullptr;
  F->keys = K;
  HFE_TRY(fs_consts(K, l, log_n_t, F->C));
  const FsConsts& C = F->C;
  const int nq = 1 << C.logn_q;
  const int64_t nt = (int64_t)nq << (log_n_t - C.logn_q);
  const int rho = C.rho, nz = C.nz, k = C.k;

  // s_T (stream TSec, element (t, 0)) and s' (stream RSec), value = (uniform mod 3) - 1
  const Mod m3 = make_mod(3);
  F->st_host.resize((size_t)nt);
  for (int64_t t = 0; t < nt; ++t)
    F->st_host[(size_t)t] = (int8_t)((int)uniform_at(seed, stream_tag(kTSec, 0), (uint64_t)t, 0, m3) - 1);
  F->sr_host.resize((size_t)nq);
  for (int t = 0; t < nq; ++t)
    F->sr_host[(size_t)t] = (int8_t)((int)uniform_at(seed, stream_tag(kRSec, 0), (uint64_t)t, 0, m3) - 1);
  HFE_TRY(put(F->st, F->st_host.data(), (size_t)nt));
  DevBuf sr;
  HFE_TRY(put(sr, F->sr_host.data(), (size_t)nq));
  HFE_TRY(put(F->cdt, K->cdt_host, sizeof(K->cdt_host)));

  // NTT(s') per slot
  DevBuf sr_hat;
  {
    std::vector<uint64_t> h((size_t)nz * nq);
    for (int z = 0; z < nz; ++z)
      for (int t = 0; t < nq; ++t) h[(size_t)z * nq + t] = residue(F->sr_host[(size_t)t], C.mod[z].q);
    HFE_TRY(put(sr_hat, h.data(), h.size() * 8));
    for (int z = 0; z < nz; ++z)
      FS_LAUNCH(launch_ntt_fwd(sr_hat.as<uint64_t>() + (size_t)z * nq, 1, nq, C.tab[z], false, nullptr));
  }
  // ring-switching keys
  {
    const size_t per_z = (size_t)(l + 1) * 2 * rho * nq;
    DevBuf coef;
    HFE_TRY(coef.alloc(per_z * nz * 8, nullptr));
    FS_LAUNCH(launch_fs_rk_coeffs(C, seed, F->st.as<int8_t>(), F->cdt.as<uint64_t>(), coef.as<uint64_t>(), nullptr));
    for (int z = 0; z < nz; ++z)
      FS_LAUNCH(launch_ntt_fwd(coef.as<uint64_t>() + z * per_z, (int64_t)(l + 1) * 2 * rho, nq, C.tab[z], false,
                               nullptr));
    HFE_TRY(F->rk.alloc(per_z * nz * 8, nullptr));
    FS_LAUNCH(launch_fs_rk_finish(C, coef.as<uint64_t>(), sr_hat.as<uint64_t>(), F->rk.as<double>(), nullptr));
    FS_LAUNCH(hipStreamSynchronize(nullptr));
  }
  // conversion keys
  {
    const size_t per_z = (size_t)(l + 1) * k * (1 + k) * nq;
    DevBuf coef;
    HFE_TRY(coef.alloc(per_z * nz * 8, nullptr));
    FS_LAUNCH(launch_fs_ck_coeffs(C, seed, sr.as<int8_t>(), F->cdt.as<uint64_t>(), coef.as<uint64_t>(), nullptr));
    for (int z = 0; z < nz; ++z)
      FS_LAUNCH(launch_ntt_fwd(coef.as<uint64_t>() + z * per_z, (int64_t)(l + 1) * k * (1 + k), nq, C.tab[z], false,
                               nullptr));
    HFE_TRY(F->ck.alloc(per_z * nz * 8, nullptr));
    FS_LAUNCH(launch_fs_ck_finish(C, coef.as<uint64_t>(), K->s_hat.as<uint64_t>(), K->L, F->ck.as<double>(), nullptr));
    FS_LAUNCH(hipStreamSynchronize(nullptr));
  }
  // transmission encryption: NTT of the polyphase parts of s_T and of Y, mod q_0 .. q_l
  {
    std::vector<uint64_t> h((size_t)(l + 1) * rho * nq);
    for (int i = 0; i <= l; ++i)
      for (int r = 0; r < rho; ++r)
        for (int u = 0; u < nq; ++u)
          h[((size_t)i * rho + r) * nq + u] = residue(F->st_host[(size_t)u * rho + r], C.mod[i].q);
    HFE_TRY(put(F->st_hat, h.data(), h.size() * 8));
    for (int i = 0; i <= l; ++i)
      FS_LAUNCH(launch_ntt_fwd(F->st_hat.as<uint64_t>() + (size_t)i * rho * nq, rho, nq, C.tab[i], false, nullptr));
    std::vector<uint64_t> y((size_t)(l + 1) * nq, 0);
    for (int i = 0; i <= l; ++i) y[(size_t)i * nq + 1] = 1;
    HFE_TRY(put(F->y_hat, y.data(), y.size() * 8));
    for (int i = 0; i <= l; ++i)
      FS_LAUNCH(launch_ntt_fwd(F->y_hat.as<uint64_t>() + (size_t)i * nq, 1, nq, C.tab[i], false, nullptr));
  }
  FS_LAUNCH(hipStreamSynchronize(nullptr));
  return HFE_OK;
}

template <class T>
T* handle_of(const void* h, uint32_t kind) {
  if (!h) return nullptr;
  const HandleBase* b = static_cast<const HandleBase*>(h);
  return b->kind == kind ? static_cast<T*>(const_cast<void*>(h)) : nullptr;
}

}  // namespace
}  // namespace hfe

using namespace hfe;

extern "C" {

hfe_status hfe_fs_keygen(const hfe_keys* keys, uint32_t level, uint32_t log_n_t, uint64_t seed, hfe_fskeys** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_keys* K = handle_of<hfe_keys>(keys, kKeys);
  if (!K) return fail(HFE_EINVAL, "invalid keys");
  if (K->family != 0) return fail(HFE_EINVAL, "FormatSwitch takes keys of the prime family");
  if (K->P.log_n_q < 6 || K->P.log_n_q > (uint32_t)kMaxLogN)
    return fail(HFE_EINVAL, "FormatSwitch needs 6 <= log_n_q <= 14");
  if (log_n_t < K->P.log_n_q || log_n_t > (uint32_t)kMaxLogNBig)
    return fail(HFE_EINVAL, "log_n_t must lie in [log_n_q, 16]");
  if (level < 1 || (int)level + 1 > K->L)
    return fail(HFE_ELEVEL, "level must be 1 .. n_q_primes - 1 (the transmission takes one prime more)");
  if (delta_log(K, (int)level) < 1) return fail(HFE_ELEVEL, "the level's modulus leaves no room for the scale");
  hfe_fskeys* F = new (std::nothrow) hfe_fskeys();
  if (!F) return fail(HFE_ENOMEM, "host allocation failed");
  hfe_status st = fs_keygen_impl(K, (int)level, (int)log_n_t, seed, F);
  if (st != HFE_OK) {
    delete F;
    return st;
  }
  *out = F;
  return HFE_OK;
}

hfe_status hfe_fs_transmit_count(const hfe_fskeys* fk, int64_t d3, int64_t* count) {
  const hfe_fskeys* F = handle_of<hfe_fskeys>(fk, kFsKeys);
  if (!F || !count) return fail(HFE_EINVAL, "invalid FormatSwitch keys or count");
  if (d3 < 0 || d3 > (1 << 20)) return fail(HFE_ESHAPE, "d3 must be 0 .. 2^20");
  *count = (int64_t)(F->C.level + 1) * d3 * F->C.k * 2 * ((int64_t)1 << F->C.logn_t);
  return HFE_OK;
}

hfe_status hfe_fs_encrypt(const hfe_fskeys* fk, const int8_t* m_q, int64_t d3, uint64_t seed, uint64_t* T,
                          void* stream) {
  const hfe_fskeys* F = handle_of<hfe_fskeys>(fk, kFsKeys);
  if (!F || !m_q || !T) return fail(HFE_EINVAL, "invalid FormatSwitch keys, m_q or T");
  if (d3 < 1 || d3 > (1 << 20)) return fail(HFE_ESHAPE, "d3 must be 1 .. 2^20");
  const FsConsts& C = F->C;
  hipStream_t s = (hipStream_t)stream;
  TernaryCheck chk;
  HFE_TRY(check_ternary_begin(m_q, d3 * C.d2, s, chk));
  DevBuf ahat;
  HFE_TRY(ahat.alloc((size_t)d3 * C.k * (C.level + 1) * ((size_t)1 << C.logn_t) * sizeof(double), s));
  FS_LAUNCH(launch_fs_tx(C, seed, m_q, d3, F->st_hat.as<uint64_t>(), F->y_hat.as<uint64_t>(), F->cdt.as<uint64_t>(),
                         ahat.as<double>(), T, s));
  return check_ternary_end(chk, "m_q");
}

hfe_status hfe_format_switch(const hfe_fskeys* fk, const uint64_t* T, int64_t d3, void* stream, hfe_qct** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_fskeys* F = handle_of<hfe_fskeys>(fk, kFsKeys);
  if (!F || !T) return fail(HFE_EINVAL, "invalid FormatSwitch keys or T");
  if (d3 < 1 || d3 > (1 << 20)) return fail(HFE_ESHAPE, "d3 must be 1 .. 2^20");
  const FsConsts& C = F->C;
  hipStream_t s = (hipStream_t)stream;
  const int64_t nq = 1ll << C.logn_q, nt = 1ll << C.logn_t;
  const int64_t ncols = d3 * C.k;
  const int64_t n_dg = ncols * (C.level + 1) * nt;
  const int64_t n_ring = (int64_t)C.nz * ncols * nq;
  const int64_t n_aconv = (int64_t)C.nz * d3 * nq;
  const int64_t n_bconv = (int64_t)C.nz * d3 * C.k * nq;
  DevBuf work;
  HFE_TRY(work.alloc((size_t)(n_dg + 2 * n_ring + n_aconv + n_bconv) * sizeof(double), s));
  FsWork w;
  w.Dg = work.as<double>();
  w.Aring = w.Dg + n_dg;
  w.Bring = w.Aring + n_ring;
  w.Aconv = w.Bring + n_ring;
  w.Bconv = w.Aconv + n_aconv;
  hfe_qct* Q = new (std::nothrow) hfe_qct();
  if (!Q) return fail(HFE_ENOMEM, "host allocation failed");
  Q->kind = kQct;
  Q->stream = s;
  Q->keys = F->keys;
  Q->level = C.level;
  Q->d3 = d3;
  Q->K = C.d2 + nq;
  hfe_status st = Q->XT.alloc(sizeof(uint64_t) * (size_t)C.level * d3 * Q->K, s);
  hipEvent_t* ev = nullptr;
  if (st == HFE_OK && profiling()) {
    for (auto& e : Q->ev)
      if (hipEventCreate(&e) != hipSuccess) st = fail(HFE_EDEVICE, "hipEventCreate");
    ev = Q->ev;
  }
  if (st == HFE_OK) {
    hipError_t e = launch_fs_switch(C, T, d3, F->rk.as<double>(), F->ck.as<double>(), w, Q->XT.as<uint64_t>(), Q->K,
                                    s, ev);
    if (e != hipSuccess) st = hip_err(e, "launch_fs_switch");
  }
  if (st != HFE_OK) {
    delete Q;
    return st;
  }
  *out = Q;
  return HFE_OK;
}

hfe_status hfe_fs_profile_ms(const hfe_qct* q, float* ms, int32_t n) {
  const hfe_qct* Q = handle_of<hfe_qct>(q, kQct);
  if (!Q || !ms || n < 0 || n > 4) return fail(HFE_EINVAL, "invalid query, ms or n (0 .. 4)");
  if (!Q->ev[0]) return fail(HFE_EINVAL, "the query was not made by a profiled FormatSwitch");
  FS_LAUNCH(hipEventSynchronize(Q->ev[4]));
  for (int i = 0; i < n; ++i) FS_LAUNCH(hipEventElapsedTime(&ms[i], Q->ev[i], Q->ev[i + 1]));
  return HFE_OK;
}

}  // extern "C"
