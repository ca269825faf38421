// The extern "C" API of the encrypted-CCMM library: validation, handle management, device
// memory and the enqueueing of the kernels for key generation, encryption, the CCMM,
// decryption and the match decision.
#include <algorithm>
#include <cstdio>
#include <map>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hfe_internal.h"

namespace hfe {

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;
}
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }
hfe_status fail(hfe_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

static hfe_status hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? HFE_ENOMEM : HFE_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

static hfe_status hip_ok_or_fail(hipError_t e) { return e == hipSuccess ? HFE_OK : hip_fail(e, "launch"); }

#define HFE_LAUNCH(expr)                              \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(_e, #expr); \
  } while (0)

// ------------------------------------------------------------------ allocator
namespace {
std::atomic<int> g_profile{0};
std::atomic<int> g_i8_variant{-1};
constexpr int kDefaultI8Variant = 0;
std::mutex g_alloc_mu;
hfe_alloc_fn g_alloc = nullptr;
hfe_dealloc_fn g_dealloc = nullptr;
void* g_alloc_ctx = nullptr;
}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  hfe_alloc_fn a;
  void* ctx;
  {
    std::lock_guard<std::mutex> l(g_alloc_mu);
    a = g_alloc;
    ctx = g_alloc_ctx;
  }
  if (a) return a(bytes, (void*)s, ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  hfe_dealloc_fn d;
  void* ctx;
  {
    std::lock_guard<std::mutex> l(g_alloc_mu);
    d = g_dealloc;
    ctx = g_alloc_ctx;
  }
  if (d) {
    d(p, (void*)s, ctx);
    return;
  }
  (void)hipFree(p);
}

hfe_status DevBuf::alloc(size_t n, hipStream_t s) {
  reset();
  ptr = dev_alloc(n, s);
  if (!ptr) return fail(HFE_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
  bytes = n;
  stream = s;
  return HFE_OK;
}

void DevBuf::reset() {
  if (ptr) dev_free(ptr, stream);
  ptr = nullptr;
  bytes = 0;
}

// ------------------------------------------------------------------ small big-integer helpers
namespace {
using u128 = unsigned __int128;

struct Big {  // little-endian 64-bit words
  std::vector<uint64_t> w;
  explicit Big(uint64_t v = 0) : w{v} {}
  void mul(uint64_t m) {
    uint64_t carry = 0;
    for (auto& x : w) {
      u128 t = (u128)x * m + carry;
      x = (uint64_t)t;
      carry = (uint64_t)(t >> 64);
    }
    if (carry) w.push_back(carry);
  }
  int bit_length() const {
    for (int i = (int)w.size() - 1; i >= 0; --i)
      if (w[i]) return i * 64 + 64 - __builtin_clzll(w[i]);
    return 0;
  }
};

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }


// The n^2 chain: random-stream id of the modulus n^2 (the prime family uses 0..8 and 16).
uint32_t chain_stream(int32_t n) { return 256u + (uint32_t)n; }

// Garner constants of the moduli q[0..level) (pairwise coprime) and the mixed-radix digits of (Q - 1) / 2.
void garner_consts_of(const uint64_t* q, int level, uint64_t garner[HFE_MAX_QPRIMES][HFE_MAX_QPRIMES],
                      uint64_t* half_digits) {
  for (int i = 0; i < level; ++i) {
    const uint64_t qi = q[i];
    uint64_t prod = 1 % qi;
    for (int j = 0; j < i; ++j) {
      garner[i][j] = prod;  // q_0..q_{j-1} mod q_i
      prod = mulmod(prod, q[j] % qi, qi);
    }
    garner[i][i] = inv_mod(prod, qi);
  }
  // mixed-radix digits of (Q - 1) / 2: halve (q_0 - 1, ..., q_{l-1} - 1) from the top digit
  uint64_t carry = 0;
  for (int i = level - 1; i >= 0; --i) {
    const u128 cur = (u128)(q[i] - 1) + (u128)carry * q[i];
    half_digits[i] = (uint64_t)(cur / 2);
    carry = (uint64_t)(cur % 2);
  }
}
void garner_consts(const hfe_keys* k, int level, uint64_t garner[HFE_MAX_QPRIMES][HFE_MAX_QPRIMES],
                   uint64_t* half_digits) {
  garner_consts_of(k->primes, level, garner, half_digits);
}
}  // namespace

// floor(log2(q_0 ... q_{l-1})) - gap
int delta_log(const hfe_keys* k, int level) {
  Big Q(1);
  for (int i = 0; i < level; ++i) Q.mul(k->family ? k->cmod[i].q : k->primes[i]);
  return Q.bit_length() - 1 - (int)k->P.gap_bits;
}

bool profiling() { return g_profile.load() != 0; }

// ------------------------------------------------------------------ validation
static hfe_status check_params(const hfe_params* P) {
  if (!P) return fail(HFE_EINVAL, "params is NULL");
  if (P->log_n_db < 1 || P->log_n_db > (uint32_t)kMaxLogNBig || P->log_n_q < 1 ||
      P->log_n_q > (uint32_t)kMaxLogNBig)
    return fail(HFE_EINVAL, "ring degrees must be 2^1 .. 2^16");
  if (P->n_q_primes < 1 || P->n_q_primes > HFE_MAX_QPRIMES)
    return fail(HFE_EINVAL, "n_q_primes must be 1..8");
  if (P->d2 < 1 || P->d2 > (1u << 20)) return fail(HFE_EINVAL, "d2 must be 1 .. 2^20");
  if (P->max_db_rows < 1 || P->max_db_rows > (1u << 24)) return fail(HFE_EINVAL, "max_db_rows out of range");
  if (P->t_den == 0 || 2ull * P->t_num >= P->t_den) return fail(HFE_EINVAL, "threshold must satisfy 0 <= t < 1/2");
  const int logmax = (int)std::max(P->log_n_db, P->log_n_q);
  std::vector<uint64_t> all(P->q, P->q + P->n_q_primes);
  all.push_back(P->p);
  for (size_t i = 0; i < all.size(); ++i) {
    const uint64_t q = all[i];
    if (q < (1ull << 20) || q >= (1ull << 36)) return fail(HFE_EINVAL, "primes must lie in [2^20, 2^36)");
    if (!is_prime_u64(q)) return fail(HFE_EINVAL, "modulus " + std::to_string(q) + " is not prime");
    if ((q - 1) % (2ull << logmax) != 0)
      return fail(HFE_EINVAL, "prime " + std::to_string(q) + " is not 1 mod 2N");
    for (size_t j = 0; j < i; ++j)
      if (all[j] == q) return fail(HFE_EINVAL, "primes must be distinct");
  }
  // Delta >= 1 for level 1 and headroom for the largest inner product: d2 * Delta < Q / 2^(gap-1)
  Big q0(P->q[0]);
  if ((int)P->gap_bits < 2 || q0.bit_length() - 1 <= (int)P->gap_bits)
    return fail(HFE_EINVAL, "gap_bits must be >= 2 and below log2 q_0");
  if ((uint64_t)P->d2 >= (1ull << (P->gap_bits - 1)))
    return fail(HFE_EOVERFLOW, "d2 * Delta would not fit below Q/2: raise gap_bits");
  return HFE_OK;
}

template <class T>
static T* as_handle(const void* h, uint32_t kind) {
  if (!h) return nullptr;
  const HandleBase* b = static_cast<const HandleBase*>(h);
  return b->kind == kind ? static_cast<T*>(const_cast<void*>(h)) : nullptr;
}


static uint32_t* pinned_flag() {
  thread_local uint32_t* p = nullptr;
  if (!p && hipHostMalloc(reinterpret_cast<void**>(&p), sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
    p = nullptr;
  return p;
}

hfe_status check_ternary_begin(const int8_t* m, int64_t n, hipStream_t s, TernaryCheck& c) {
  c.host = pinned_flag();
  if (!c.host) return fail(HFE_ENOMEM, "pinned host allocation failed");
  HFE_TRY(c.flag.alloc(sizeof(uint32_t), s));
  HFE_LAUNCH(hipMemsetAsync(c.flag.ptr, 0, sizeof(uint32_t), s));
  HFE_LAUNCH(launch_check_ternary(m, n, c.flag.as<uint32_t>(), s));
  HFE_LAUNCH(hipMemcpyAsync(c.host, c.flag.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HFE_LAUNCH(hipEventCreateWithFlags(&c.ev, hipEventDisableTiming));
  HFE_LAUNCH(hipEventRecord(c.ev, s));
  return HFE_OK;
}

hfe_status check_ternary_end(TernaryCheck& c, const char* what) {
  HFE_LAUNCH(hipEventSynchronize(c.ev));
  if (*c.host) return fail(HFE_EINVAL, std::string(what) + " has entries outside {-1, 0, 1}");
  return HFE_OK;
}

}  // namespace hfe

using namespace hfe;

extern "C" {

const char* hfe_last_error(void) { return get_error(); }

hfe_status hfe_set_allocator(hfe_alloc_fn alloc, hfe_dealloc_fn dealloc, void* ctx) {
  if ((alloc == nullptr) != (dealloc == nullptr))
    return fail(HFE_EINVAL, "alloc and dealloc must both be set or both be NULL");
  std::lock_guard<std::mutex> l(g_alloc_mu);
  g_alloc = alloc;
  g_dealloc = dealloc;
  g_alloc_ctx = ctx;
  return HFE_OK;
}

hfe_status hfe_cdt_table(uint64_t* dst) {
  if (!dst) return fail(HFE_EINVAL, "dst is NULL");
  if (cdt_table_quad_impl(dst) != 0) return fail(HFE_EINTERNAL, "CDT table out of range");
  return HFE_OK;
}

hfe_status hfe_default_params(uint32_t log_n_db, uint32_t log_n_q, uint32_t n_q_primes, uint32_t d2,
                              uint32_t max_db_rows, hfe_params* out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  if (n_q_primes < 1 || n_q_primes > HFE_MAX_QPRIMES) return fail(HFE_EINVAL, "n_q_primes must be 1..8");
  hfe_params P;
  std::memset(&P, 0, sizeof(P));
  P.log_n_db = log_n_db;
  P.log_n_q = log_n_q;
  P.n_q_primes = n_q_primes;
  P.gap_bits = 20;
  P.d2 = d2;
  P.max_db_rows = max_db_rows;
  P.t_num = 3;
  P.t_den = 8;
  const uint64_t step = 1ull << 17;
  uint64_t c = ((1ull << 36) - 1) / step * step + 1;
  std::vector<uint64_t> primes;
  while (primes.size() < n_q_primes + 1) {
    if (is_prime_u64(c)) primes.push_back(c);
    c -= step;
  }
  P.p = primes[0];
  for (uint32_t i = 0; i < n_q_primes; ++i) P.q[i] = primes[i + 1];
  HFE_TRY(check_params(&P));
  *out = P;
  return HFE_OK;
}

// ------------------------------------------------------------------ keygen
static hfe_status upload(DevBuf& b, const void* host, size_t bytes) {
  HFE_TRY(b.alloc(bytes, nullptr));
  HFE_LAUNCH(hipMemcpy(b.ptr, host, bytes, hipMemcpyHostToDevice));
  return HFE_OK;
}

static hfe_status keygen_impl(const hfe_params* params, uint64_t seed, hfe_keys* K) {
  K->kind = kKeys;
  K->stream = nullptr;
  K->P = *params;
  const hfe_params& P = K->P;
  K->L = (int)P.n_q_primes;
  K->n_primes = K->L + 1;
  for (int i = 0; i < K->L; ++i) {
    K->primes[i] = P.q[i];
    K->prime_id[i] = (uint32_t)i;
  }
  K->primes[K->L] = P.p;
  K->prime_id[K->L] = kPrimeIdP;
  for (int i = 0; i < K->n_primes; ++i) K->mods[i] = make_mod(K->primes[i]);
  const int nq = 1 << P.log_n_q, ndb = 1 << P.log_n_db;
  K->k = (int)((P.d2 + nq - 1) / nq);
  K->k_db = (int)((P.max_db_rows + ndb - 1) / ndb);

  // ternary secrets (streams QSEC / DBSEC, element (t, 0)), value = (uniform mod 3) - 1
  const Mod m3 = make_mod(3);
  K->s_host.resize((size_t)K->k * nq);
  for (int j = 0; j < K->k; ++j)
    for (int t = 0; t < nq; ++t)
      K->s_host[(size_t)j * nq + t] = (int8_t)((int)uniform_at(seed, stream_tag(kQSec, j), t, 0, m3) - 1);
  K->sdb_host.resize((size_t)K->k_db * ndb);
  for (int j = 0; j < K->k_db; ++j)
    for (int t = 0; t < ndb; ++t)
      K->sdb_host[(size_t)j * ndb + t] = (int8_t)((int)uniform_at(seed, stream_tag(kDbSec, j), t, 0, m3) - 1);

  // twiddle tables
  std::vector<uint64_t> tab;
  for (int z = 0; z < K->n_primes; ++z) {
    const uint64_t q = K->primes[z];
    for (int which = 0; which < 2; ++which) {
      const int logn = which == 0 ? (int)P.log_n_db : (int)P.log_n_q;
      NttTabOwner& o = which == 0 ? K->tab_db[z] : K->tab_q[z];
      ntt_tables_host(q, logn, tab);  // psi | psi_sh | ipsi | ipsi_sh
      const size_t n = (size_t)1 << logn;
      // the transforms take the twiddles as doubles (exact: below 2^36)
      std::vector<double> td(2 * n);
      for (size_t i = 0; i < n; ++i) {
        td[i] = (double)tab[i];
        td[n + i] = (double)tab[2 * n + i];
      }
      HFE_TRY(upload(o.buf, td.data(), td.size() * sizeof(double)));
      const double* base = o.buf.as<double>();
      o.tab.psi_d = base;
      o.tab.ipsi_d = base + n;
      o.tab.q = q;
      o.tab.qd = (double)q;
      o.tab.qinv = 1.0 / (double)q;  // correctly rounded
      o.tab.n_inv_d = (double)inv_mod(n % q, q);
      o.tab.logn = logn;
    }
  }

  // NTT-domain secrets with Shoup companions: blocks of [n values | n companions]
  auto residue = [](int v, uint64_t q) -> uint64_t { return v >= 0 ? (uint64_t)v : q - (uint64_t)(-v); };
  {
    std::vector<uint64_t> h((size_t)K->n_primes * K->k * 2 * nq, 0);
    for (int z = 0; z < K->n_primes; ++z)
      for (int j = 0; j < K->k; ++j)
        for (int t = 0; t < nq; ++t)
          h[(((size_t)z * K->k + j) * 2) * nq + t] = residue(K->s_host[(size_t)j * nq + t], K->primes[z]);
    HFE_TRY(upload(K->s_hat, h.data(), h.size() * 8));
    for (int z = 0; z < K->n_primes; ++z)
      HFE_LAUNCH(launch_ntt_fwd(K->s_hat.as<uint64_t>() + (size_t)z * K->k * 2 * nq, K->k, 2 * nq,
                                K->tab_q[z].tab, true, nullptr));
  }
  {
    // s~_j(X) = s_j(1/X) = s_0 - sum_{t>=1} s_{n-t} X^t, mod q_0 (T = M_DB S_Q is exact there)
    std::vector<uint64_t> h((size_t)K->k * 2 * nq, 0);
    for (int j = 0; j < K->k; ++j)
      for (int t = 0; t < nq; ++t) {
        const int v = t == 0 ? K->s_host[(size_t)j * nq] : -K->s_host[(size_t)j * nq + nq - t];
        h[(size_t)j * 2 * nq + t] = residue(v, K->primes[0]);
      }
    HFE_TRY(upload(K->sconj_hat, h.data(), h.size() * 8));
    HFE_LAUNCH(launch_ntt_fwd(K->sconj_hat.as<uint64_t>(), K->k, 2 * nq, K->tab_q[0].tab, true, nullptr));
  }
  {
    std::vector<uint64_t> h((size_t)K->n_primes * K->k_db * 2 * ndb, 0);
    for (int z = 0; z < K->n_primes; ++z)
      for (int j = 0; j < K->k_db; ++j)
        for (int t = 0; t < ndb; ++t)
          h[(((size_t)z * K->k_db + j) * 2) * ndb + t] =
              residue(K->sdb_host[(size_t)j * ndb + t], K->primes[z]);
    HFE_TRY(upload(K->sdb_hat, h.data(), h.size() * 8));
    for (int z = 0; z < K->n_primes; ++z)
      HFE_LAUNCH(launch_ntt_fwd(K->sdb_hat.as<uint64_t>() + (size_t)z * K->k_db * 2 * ndb, K->k_db,
                                2 * ndb, K->tab_db[z].tab, true, nullptr));
  }
  if (cdt_table_quad_impl(K->cdt_host) != 0) return fail(HFE_EINTERNAL, "CDT table out of range");
  HFE_TRY(upload(K->cdt, K->cdt_host, sizeof(K->cdt_host)));
  HFE_LAUNCH(hipDeviceSynchronize());
  return HFE_OK;
}

hfe_status hfe_keygen(const hfe_params* params, uint64_t seed, hfe_keys** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  HFE_TRY(check_params(params));
  hfe_keys* K = new (std::nothrow) hfe_keys();
  if (!K) return fail(HFE_ENOMEM, "host allocation failed");
  hfe_status st = keygen_impl(params, seed, K);
  if (st != HFE_OK) {
    delete K;
    return st;
  }
  *out = K;
  return HFE_OK;
}

// ------------------------------------------------------------------ encode
hfe_status hfe_chain_default_params(uint32_t log_n_db, uint32_t log_n_q, uint32_t n_q_mods, uint32_t n_p_mods,
                                    uint32_t d2, uint32_t max_db_rows, hfe_chain_params* out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  if (n_q_mods < 1 || n_q_mods > HFE_MAX_QPRIMES || n_p_mods < 1 || n_p_mods > (uint32_t)kChainMaxP)
    return fail(HFE_EINVAL, "n_q_mods must be 1..8 and n_p_mods 1..3");
  hfe_chain_params C;
  std::memset(&C, 0, sizeof(C));
  C.log_n_db = log_n_db;
  C.log_n_q = log_n_q;
  C.n_q_mods = n_q_mods;
  C.n_p_mods = n_p_mods;
  uint32_t k = 0;
  for (uint32_t n = 253; n >= 127 && k < n_q_mods + n_p_mods; --n)
    if (is_prime_u64(n)) C.bases[k++] = n;
  const uint64_t step = 1ull << 17;
  uint64_t c = ((1ull << 36) - 1) / step * step + 1;
  while (!is_prime_u64(c)) c -= step;
  C.ntt_prime = c;
  C.gap_bits = 20;
  C.d2 = d2;
  C.max_db_rows = max_db_rows;
  C.t_num = 3;
  C.t_den = 8;
  *out = C;
  return HFE_OK;
}

hfe_status hfe_chain_keygen(const hfe_chain_params* C, uint64_t seed, hfe_keys** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!C) return fail(HFE_EINVAL, "params is NULL");
  if (C->n_q_mods < 1 || C->n_q_mods > HFE_MAX_QPRIMES || C->n_p_mods < 1 || C->n_p_mods > (uint32_t)kChainMaxP)
    return fail(HFE_EINVAL, "n_q_mods must be 1..8 and n_p_mods 1..3");
  const int nm = (int)(C->n_q_mods + C->n_p_mods);
  for (int i = 0; i < nm; ++i) {
    const uint32_t n = C->bases[i];
    if (n < 127 || n > 253 || !is_prime_u64(n)) return fail(HFE_EINVAL, "chain bases must be primes in [127, 253]");
    for (int j = 0; j < i; ++j)
      if (C->bases[j] == n) return fail(HFE_EINVAL, "chain bases must be distinct");
  }
  // the secrets and the tables of the NTT prime come from the prime family's key generation, with
  // the NTT prime as q_0 and another prime = 1 mod 2^17 as p (its tables are not used)
  hfe_params P;
  std::memset(&P, 0, sizeof(P));
  P.log_n_db = C->log_n_db;
  P.log_n_q = C->log_n_q;
  P.n_q_primes = 1;
  P.q[0] = C->ntt_prime;
  const uint64_t step = 1ull << 17;
  uint64_t c = ((1ull << 36) - 1) / step * step + 1;
  while (c == C->ntt_prime || !is_prime_u64(c)) c -= step;
  P.p = c;
  P.gap_bits = C->gap_bits;
  P.d2 = C->d2;
  P.max_db_rows = C->max_db_rows;
  P.t_num = C->t_num;
  P.t_den = C->t_den;
  HFE_TRY(check_params(&P));
  hfe_keys* K = new (std::nothrow) hfe_keys();
  if (!K) return fail(HFE_ENOMEM, "host allocation failed");
  hfe_status st = keygen_impl(&P, seed, K);
  if (st != HFE_OK) {
    delete K;
    return st;
  }
  K->family = 1;
  K->cq = (int)C->n_q_mods;
  K->cp = (int)C->n_p_mods;
  K->cP = 1;
  for (int i = 0; i < nm; ++i) {
    K->cbase[i] = (int32_t)C->bases[i];
    K->cmod[i] = make_mod((uint64_t)C->bases[i] * C->bases[i]);
    if (i >= K->cq) K->cP *= K->cmod[i].q;
  }
  *out = K;
  return HFE_OK;
}

hfe_status hfe_encode(const uint8_t* codes, const uint8_t* masks, int64_t n, int32_t d2,
                      const int32_t* shifts, int32_t n_shifts, int8_t* out, void* stream) {
  if (!codes || !masks || !shifts || !out) return fail(HFE_EINVAL, "NULL argument");
  if (n < 0 || d2 < 1) return fail(HFE_ESHAPE, "bad sizes");
  if (n_shifts < 1 || n_shifts > 64) return fail(HFE_EINVAL, "n_shifts must be 1..64");
  HFE_LAUNCH(launch_encode(codes, masks, n, d2, shifts, n_shifts, out, (hipStream_t)stream));
  return HFE_OK;
}

// ------------------------------------------------------------------ database encryption
// Small moduli of the RNS form for contraction length K: the shortest prefix of kRnsMods whose
// product M is at least 4 K h^2 (h = (q - 1) / 2 for the largest prime of the basis): the
// centered sum S of K products of centered residues is determined by S mod M, with |S| <= M / 4
// so that the CRT can round its multiple of M from a single-precision sum.  K < 2^17 keeps every
// int32 accumulation of int8 products exact.
static hfe_status rns_moduli_for(const hfe_keys* K, int64_t Klen, int* n_out) {
  if (Klen >= (1 << 17)) return fail(HFE_ESHAPE, "RNS form: contraction length must be below 2^17");
  uint64_t qmax = 0;
  for (int z = 0; z < K->n_primes; ++z) qmax = std::max(qmax, K->primes[z]);
  const unsigned __int128 h = (qmax - 1) / 2;
  const unsigned __int128 bound = (unsigned __int128)4 * (uint64_t)Klen * h * h;
  unsigned __int128 M = 1;
  for (int n = 1; n <= kRnsMaxMods; ++n) {
    M *= (uint64_t)kRnsMods[n - 1];
    if (M >= bound) {
      *n_out = n;
      return HFE_OK;
    }
  }
  return fail(HFE_ESHAPE, "RNS form: contraction too long for the small moduli");
}

// a^-1 mod m for gcd(a, m) = 1 (extended Euclid; m need not be prime).
static int64_t inv_mod_any(int64_t a, int64_t m) {
  int64_t r0 = m, r1 = ((a % m) + m) % m, t0 = 0, t1 = 1;
  while (r1 != 0) {
    const int64_t qt = r0 / r1;
    const int64_t r2 = r0 - qt * r1, t2 = t0 - qt * t1;
    r0 = r1;
    r1 = r2;
    t0 = t1;
    t1 = t2;
  }
  return ((t0 % m) + m) % m;  // r0 == 1 for coprime inputs
}

// CRT constants of the RNS form: (M/m_j)^-1 mod m_j, 1/m_j, and (M/m_j), M mod the prime of each
// slot of a level.
static RnsCrtArgs make_rns_crt_args(const hfe_keys* K, int level, int n) {
  RnsCrtArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  ra.n = n;
  unsigned __int128 M = 1;
  for (int i = 0; i < n; ++i) M *= (uint64_t)kRnsMods[i];
  for (int j = 0; j < n; ++j) {
    const int64_t m = kRnsMods[j];
    ra.m[j] = (int32_t)m;
    ra.magic[j] = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)m - 1) / (uint64_t)m);
    const unsigned __int128 Mj = M / (uint64_t)m;
    ra.inv[j] = (int32_t)inv_mod_any((int64_t)(Mj % (uint64_t)m), m);
    ra.rcp[j] = 1.0f / (float)m;
  }
  for (int z = 0; z <= level; ++z) {
    const int slot = z < level ? z : K->L;
    const uint64_t q = K->primes[slot];
    ra.mod[z] = K->mods[slot];
    ra.M_mod_q[z] = (uint64_t)(M % q);
    for (int j = 0; j < n; ++j) ra.Mj_mod_q[z][j] = (uint64_t)((M / (uint64_t)kRnsMods[j]) % q);
  }
  return ra;
}

// Bases of the n^2 form for contraction length K: the shortest prefix of kP2Bases whose squares'
// product M is at least 4 K h^2 (as for the RNS form).  K <= 2^16 keeps the int32 accumulation of
// the 2 K products of each G1 sum exact (|digits| <= 125).
static hfe_status p2_bases_for(const hfe_keys* K, int64_t Klen, int* n_out) {
  if (Klen > (1 << 16)) return fail(HFE_ESHAPE, "n^2 form: contraction length must be at most 2^16");
  uint64_t qmax = 0;
  for (int z = 0; z < K->n_primes; ++z) qmax = std::max(qmax, K->primes[z]);
  const unsigned __int128 h = (qmax - 1) / 2;
  const unsigned __int128 bound = (unsigned __int128)4 * (uint64_t)Klen * h * h;
  unsigned __int128 M = 1;
  for (int n = 1; n <= kP2MaxBases; ++n) {
    M *= (uint64_t)kP2Bases[n - 1] * (uint64_t)kP2Bases[n - 1];
    if (M >= bound) {
      *n_out = n;
      return HFE_OK;
    }
  }
  return fail(HFE_ESHAPE, "n^2 form: contraction too long for the bases");
}

// CRT constants of the n^2 form (moduli m_j = n_j^2), as make_rns_crt_args.
static P2CrtArgs make_p2_crt_args(const hfe_keys* K, int level, int n) {
  P2CrtArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  ra.n = n;
  unsigned __int128 M = 1;
  for (int i = 0; i < n; ++i) M *= (uint64_t)kP2Bases[i] * (uint64_t)kP2Bases[i];
  for (int j = 0; j < n; ++j) {
    const int64_t m = (int64_t)kP2Bases[j] * kP2Bases[j];
    ra.m[j] = (int32_t)m;
    const unsigned __int128 Mj = M / (uint64_t)m;
    ra.inv[j] = (int32_t)inv_mod_any((int64_t)(Mj % (uint64_t)m), m);
    ra.rcp[j] = 1.0f / (float)m;
  }
  for (int z = 0; z <= level; ++z) {
    const int slot = z < level ? z : K->L;
    const uint64_t q = K->primes[slot];
    ra.mod[z] = K->mods[slot];
    ra.M_mod_q[z] = (uint64_t)(M % q);
    for (int j = 0; j < n; ++j) ra.Mj_mod_q[z][j] = (uint64_t)((M / (uint64_t)ra.m[j]) % q);
  }
  return ra;
}

// The database over the n^2 chain: T through the NTT prime, then for each modulus (query moduli,
// then the special part's) the encryption with scale P and the split into that modulus' slot of
// the n^2 planes (special moduli first).  The plain form keeps every modulus' residues.
static hfe_status chain_encrypt_db_impl(const hfe_keys* K, const int8_t* m_db, int64_t d1, uint64_t seed,
                                        uint32_t forms, hipStream_t s, hfe_db* D) {
  const hfe_params& P = K->P;
  const int64_t ndb = 1ll << P.log_n_db, nq = 1ll << P.log_n_q;
  if (!(forms & HFE_FORM_P2_I8) || (forms & ~(uint32_t)(HFE_FORM_P2_I8 | HFE_FORM_PLAIN_U64)))
    return fail(HFE_EINVAL, "the n^2 modulus chain takes HFE_FORM_P2_I8 (and HFE_FORM_PLAIN_U64 to keep residues)");
  D->kind = kDb;
  D->stream = s;
  D->keys = K;
  D->d1 = d1;
  D->R = ndb + d1;
  D->K = (int64_t)P.d2 + nq;
  if (D->K > (1ll << 16)) return fail(HFE_ESHAPE, "the n^2 contraction needs d2 + N_Q <= 2^16");
  D->KB = (D->K + kKB - 1) / kKB;
  D->R_pad = (D->R + 63) / 64 * 64 + kRowPad;
  D->forms = forms;
  const int nm = K->cq + K->cp;
  D->slots_plain = nm;
  D->slots_planes = 1;
  D->n_p2 = nm;
  DevBuf MT, Trow, Tt;
  HFE_TRY(MT.alloc((size_t)P.d2 * d1, s));
  HFE_TRY(Trow.alloc(sizeof(int32_t) * (size_t)nq * d1, s));
  HFE_TRY(Tt.alloc(sizeof(int32_t) * (size_t)nq * d1, s));
  HFE_LAUNCH(launch_transpose_i8(m_db, d1, P.d2, MT.as<int8_t>(), s));
  HFE_LAUNCH(launch_db_T(m_db, d1, (int32_t)P.d2, K->sconj_hat.as<uint64_t>(), K->k, K->tab_q[0].tab,
                         Trow.as<int32_t>(), Tt.as<int32_t>(), s));
  const bool keep_plain = (forms & HFE_FORM_PLAIN_U64) != 0;
  const size_t prime_elems = (size_t)D->K * D->R;
  DevBuf one;
  if (keep_plain)
    HFE_TRY(D->Dt.alloc(sizeof(uint64_t) * (size_t)nm * prime_elems, s));
  else
    HFE_TRY(one.alloc(sizeof(uint64_t) * prime_elems, s));
  const size_t plane = (size_t)D->KB * D->R_pad * kKB;
  HFE_TRY(D->p2.alloc((size_t)nm * 2 * plane, s));
  DbEncArgs a;
  a.seed = seed;
  a.MT = MT.as<int8_t>();
  a.Tt = Tt.as<int32_t>();
  a.cdt = K->cdt.as<uint64_t>();
  a.d1 = d1;
  a.d2 = P.d2;
  a.K = D->K;
  a.R = D->R;
  a.k_db = K->k_db;
  a.p = K->cP;
  for (int i = 0; i < nm; ++i) {
    uint64_t* Di = keep_plain ? D->Dt.as<uint64_t>() + (size_t)i * prime_elems : one.as<uint64_t>();
    HFE_LAUNCH(launch_db_encrypt(a, Di, chain_stream(K->cbase[i]), K->cmod[i], K->tab_db[0].tab,
                                 K->sdb_hat.as<uint64_t>(), s));
    const int slot = i < K->cq ? K->cp + i : i - K->cq;
    HFE_LAUNCH(launch_chain_split_db(Di, D->K, D->R, D->KB, D->R_pad, chain_base(K->cbase[i]),
                                     D->p2.as<int8_t>() + (size_t)slot * 2 * plane, s));
  }
  return HFE_OK;
}

static hfe_status encrypt_db_impl(const hfe_keys* K, const int8_t* m_db, int64_t d1, uint64_t seed,
                                  uint32_t forms, hipStream_t s, hfe_db* D) {
  if (K->family) return chain_encrypt_db_impl(K, m_db, d1, seed, forms, s, D);
  const hfe_params& P = K->P;
  const int64_t ndb = 1ll << P.log_n_db, nq = 1ll << P.log_n_q;
  D->kind = kDb;
  D->stream = s;
  D->keys = K;
  D->d1 = d1;
  D->R = ndb + d1;
  D->K = (int64_t)P.d2 + nq;
  D->KB = (D->K + kKB - 1) / kKB;
  D->R_pad = (D->R + 63) / 64 * 64 + kRowPad;
  D->forms = forms;
  const int np = K->n_primes;
  D->slots_plain = D->slots_planes = np;

  DevBuf MT, Trow, Tt;
  HFE_TRY(MT.alloc((size_t)P.d2 * d1, s));
  HFE_TRY(Trow.alloc(sizeof(int32_t) * (size_t)nq * d1, s));
  HFE_TRY(Tt.alloc(sizeof(int32_t) * (size_t)nq * d1, s));
  HFE_LAUNCH(launch_transpose_i8(m_db, d1, P.d2, MT.as<int8_t>(), s));
  HFE_LAUNCH(launch_db_T(m_db, d1, (int32_t)P.d2, K->sconj_hat.as<uint64_t>(), K->k, K->tab_q[0].tab,
                         Trow.as<int32_t>(), Tt.as<int32_t>(), s));
  // With the plain form kept, every prime's residues stay in D->Dt.  Otherwise one prime at a time
  // is encrypted into a scratch buffer and split into the int8 forms' planes, so the residues of
  // all primes (8 bytes per entry and prime) never need to be resident at once.
  const bool keep_plain = (forms & HFE_FORM_PLAIN_U64) != 0;
  const size_t prime_elems = (size_t)D->K * D->R;
  DevBuf one;
  if (keep_plain)
    HFE_TRY(D->Dt.alloc(sizeof(uint64_t) * (size_t)np * prime_elems, s));
  else
    HFE_TRY(one.alloc(sizeof(uint64_t) * prime_elems, s));
  const size_t plane = (size_t)D->KB * D->R_pad * kKB;
  if (forms & HFE_FORM_I8_MFMA) HFE_TRY(D->digits.alloc((size_t)np * kDigits * plane, s));
  if (forms & HFE_FORM_RNS_I8) {
    int n = 0;
    HFE_TRY(rns_moduli_for(K, D->K, &n));
    D->n_rns = n;
    HFE_TRY(D->rns.alloc((size_t)np * n * plane, s));
  }
  if (forms & HFE_FORM_P2_I8) {
    int n = 0;
    HFE_TRY(p2_bases_for(K, D->K, &n));
    D->n_p2 = n;
    HFE_TRY(D->p2.alloc((size_t)np * 2 * n * plane, s));
  }
  DbEncArgs a;
  a.seed = seed;
  a.MT = MT.as<int8_t>();
  a.Tt = Tt.as<int32_t>();
  a.cdt = K->cdt.as<uint64_t>();
  a.d1 = d1;
  a.d2 = P.d2;
  a.K = D->K;
  a.R = D->R;
  a.k_db = K->k_db;
  a.p = P.p;
  for (int z = 0; z < np; ++z) {
    uint64_t* Dz = keep_plain ? D->Dt.as<uint64_t>() + (size_t)z * prime_elems : one.as<uint64_t>();
    HFE_LAUNCH(launch_db_encrypt(a, Dz, K->prime_id[z], K->mods[z], K->tab_db[z].tab,
                                 K->sdb_hat.as<uint64_t>() + (size_t)z * K->k_db * 2 * ndb, s));
    if (forms & HFE_FORM_I8_MFMA)
      HFE_LAUNCH(launch_split_db(Dz, D->K, D->R, D->KB, D->R_pad, K->primes[z],
                                 D->digits.as<int8_t>() + (size_t)z * kDigits * plane, s));
    if (forms & HFE_FORM_RNS_I8)
      HFE_LAUNCH(launch_split_db_rns(Dz, D->K, D->R, D->KB, D->R_pad, K->primes[z], D->n_rns,
                                     D->rns.as<int8_t>() + (size_t)z * D->n_rns * plane, s));
    if (forms & HFE_FORM_P2_I8)
      HFE_LAUNCH(launch_split_db_p2(Dz, D->K, D->R, D->KB, D->R_pad, K->primes[z], D->n_p2,
                                    D->p2.as<int8_t>() + (size_t)z * 2 * D->n_p2 * plane, s));
  }
  return HFE_OK;
}

hfe_status hfe_encrypt_db(const hfe_keys* keys, const int8_t* m_db, int64_t d1, uint64_t seed, uint32_t forms,
                          void* stream, hfe_db** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_keys* K = as_handle<hfe_keys>(keys, kKeys);
  if (!K || !m_db) return fail(HFE_EINVAL, "invalid keys or m_db");
  if (d1 < 1 || d1 > (int64_t)K->P.max_db_rows)
    return fail(HFE_ESHAPE, "d1 must be 1 .. max_db_rows");
  if (forms == 0 || (forms & ~15u)) return fail(HFE_EINVAL, "forms must be a non-empty set of hfe_form");
  TernaryCheck chk;
  HFE_TRY(check_ternary_begin(m_db, d1 * (int64_t)K->P.d2, (hipStream_t)stream, chk));
  hfe_db* D = new (std::nothrow) hfe_db();
  if (!D) return fail(HFE_ENOMEM, "host allocation failed");
  hfe_status st = encrypt_db_impl(K, m_db, d1, seed, forms, (hipStream_t)stream, D);
  if (st == HFE_OK) st = check_ternary_end(chk, "m_db");  // a refused input: buffers freed in stream order
  if (st != HFE_OK) {
    delete D;
    return st;
  }
  *out = D;
  return HFE_OK;
}

// ------------------------------------------------------------------ query encryption
hfe_status hfe_encrypt(const hfe_keys* keys, const int8_t* m_q, int64_t d3, uint32_t level, uint64_t seed,
                       void* stream, hfe_qct** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_keys* K = as_handle<hfe_keys>(keys, kKeys);
  if (!K || !m_q) return fail(HFE_EINVAL, "invalid keys or m_q");
  if (d3 < 1 || d3 > (1 << 20)) return fail(HFE_ESHAPE, "d3 must be 1 .. 2^20");
  if (level < 1 || (int)level > (K->family ? K->cq : K->L)) return fail(HFE_ELEVEL, "level must be 1 .. n_q_primes");
  if (delta_log(K, (int)level) < 1) return fail(HFE_ELEVEL, "the level's modulus leaves no room for the scale");
  hipStream_t s = (hipStream_t)stream;
  const hfe_params& P = K->P;
  TernaryCheck chk;
  HFE_TRY(check_ternary_begin(m_q, d3 * (int64_t)P.d2, s, chk));
  const int64_t nq = 1ll << P.log_n_q;
  hfe_qct* Q = new (std::nothrow) hfe_qct();
  if (!Q) return fail(HFE_ENOMEM, "host allocation failed");
  Q->kind = kQct;
  Q->stream = s;
  Q->keys = K;
  Q->level = (int)level;
  Q->d3 = d3;
  Q->K = (int64_t)P.d2 + nq;
  hfe_status st = Q->XT.alloc(sizeof(uint64_t) * (size_t)level * d3 * Q->K, s);
  if (st != HFE_OK) {
    delete Q;
    return st;
  }
  QEncArgs a;
  a.seed = seed;
  a.m_q = m_q;
  a.cdt = K->cdt.as<uint64_t>();
  a.d3 = d3;
  a.d2 = P.d2;
  a.K = Q->K;
  a.k = K->k;
  // the errors are the same integers for every prime: drawn once when more than one prime needs them
  // (the LDS-resident transforms; the two-pass ones draw their own)
  DevBuf errs;
  if (level > 1 && P.log_n_q <= (uint32_t)kMaxLogN) {
    st = errs.alloc((size_t)d3 * P.d2, s);
    if (st == HFE_OK) {
      const hipError_t e = launch_q_errors(seed, a.cdt, d3, P.d2, errs.as<int8_t>(), s);
      if (e != hipSuccess) st = hip_fail(e, "launch_q_errors");
    }
    if (st != HFE_OK) {
      delete Q;
      return st;
    }
    a.e = errs.as<int8_t>();
  }
  const int dl = delta_log(K, (int)level);
  for (uint32_t i = 0; i < level; ++i) {
    // the n^2 chain: modulus n_i^2, products with the secrets through the NTT prime (slot 0)
    const bool ch = K->family != 0;
    const Mod& md = ch ? K->cmod[i] : K->mods[i];
    const uint64_t delta_mod = pow_mod(2, (uint64_t)dl, md.q);
    hipError_t e = launch_q_encrypt(a, Q->XT.as<uint64_t>() + (size_t)i * d3 * Q->K,
                                    ch ? chain_stream(K->cbase[i]) : K->prime_id[i], md, delta_mod,
                                    K->tab_q[ch ? 0 : i].tab,
                                    K->s_hat.as<uint64_t>() + (size_t)(ch ? 0 : i) * K->k * 2 * nq, s);
    if (e != hipSuccess) {
      delete Q;
      return hip_fail(e, "launch_q_encrypt");
    }
  }
  st = check_ternary_end(chk, "m_q");  // a refused input: the ciphertext is freed in stream order
  if (st != HFE_OK) {
    delete Q;
    return st;
  }
  *out = Q;
  return HFE_OK;
}

// ------------------------------------------------------------------ CCMM
static LiftArgs make_lift_args(const hfe_keys* K, int level) {
  LiftArgs la;
  std::memset(&la, 0, sizeof(la));
  la.level = level;
  for (int i = 0; i < level; ++i) {
    la.q[i] = K->primes[i];
    la.mu[i] = K->mods[i].mu;
  }
  la.p = K->P.p;
  la.mu_p = K->mods[K->L].mu;
  garner_consts(K, level, la.garner, la.half_digits);
  uint64_t prod = 1;
  for (int i = 0; i < level; ++i) {
    la.mprod_p[i] = prod;
    prod = mulmod(prod, K->primes[i] % K->P.p, K->P.p);
  }
  la.mprod_p[level] = prod;
  la.Q_mod_p = prod;
  return la;
}

static RescaleArgs make_rescale_args(const hfe_keys* K, int level) {
  RescaleArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  ra.level = level;
  ra.p = K->P.p;
  for (int i = 0; i < level; ++i) {
    ra.mod[i] = K->mods[i];
    ra.pinv[i] = inv_mod(K->P.p % K->primes[i], K->primes[i]);
    ra.pinv_sh[i] = shoup(ra.pinv[i], K->primes[i]);
  }
  return ra;
}

// Autotuned tile configurations: (level, d3 bucket) -> variant.
static std::mutex g_tune_mu;
static std::map<std::pair<int, int64_t>, int> g_tuned;
static int64_t d3_bucket(int64_t d3) {
  int64_t b = 64;
  while (b < d3) b <<= 1;
  return b;
}
// The forced variant if one is set; else the tuned entry of this level with the nearest column
// bucket; else the default.
static int pick_i8_variant(int level, int64_t d3) {
  const int forced = g_i8_variant.load();
  if (forced >= 0) return forced;
  std::lock_guard<std::mutex> l(g_tune_mu);
  const int64_t b = d3_bucket(d3);
  int best = kDefaultI8Variant;
  int64_t best_dist = -1;
  for (const auto& kv : g_tuned) {
    if (kv.first.first != level) continue;
    const int64_t dist = kv.first.second > b ? kv.first.second / b : b / kv.first.second;
    if (best_dist < 0 || dist < best_dist) {
      best_dist = dist;
      best = kv.second;
    }
  }
  return best;
}

// Device buffers of one call: from the allocator (released in stream order when the workspace goes
// out of scope), or carved from a caller-provided region (the allocation-free entry point), each at
// a 256-byte boundary; a request beyond the region's end fails with HFE_ENOMEM before anything is
// enqueued for it.
extern "C++" {
struct Workspace {
  uint8_t* base = nullptr;  // region mode when set
  size_t cap = 0, used = 0;
  DevBuf bufs[4];
  int nb = 0;
  template <class T>
  hfe_status get(size_t bytes, hipStream_t s, T** out) {
    if (base) {
      const size_t off = (used + 255) & ~(size_t)255;
      if (off > cap || bytes > cap - off)
        return fail(HFE_ENOMEM, "the call needs more scratch than the " + std::to_string(cap) + "-byte region");
      *out = reinterpret_cast<T*>(base + off);
      used = off + bytes;
      return HFE_OK;
    }
    if (nb == 4) return fail(HFE_EINTERNAL, "workspace: too many buffers");
    HFE_TRY(bufs[nb].alloc(bytes, s));
    *out = bufs[nb++].as<T>();
    return HFE_OK;
  }
};
}  // extern "C++"

// Every buffer of the call is obtained before its first launch, so a workspace that cannot supply
// one fails the call with nothing enqueued.
// C_ext == nullptr: the result (rescaled residues) into R->out.  C_ext != nullptr: only the exact
// product before the rescale, C_ext[z][c][r] for the level's primes and p (z = level), and R only
// records the shape.
// out_ext != nullptr: the result into that caller-owned buffer instead of R->out.  ws: where the
// call's buffers come from (nullptr: the allocator).
// The CCMM over the n^2 chain (Section 6.3): lift the query from Q_l to the special moduli and split
// every slot into M, M'; one n^2 contraction launch over the slots [0, cp + l) (three int8 products
// per modulus, residues mod n^2 directly); RS_P into the result [l][d3][N_DB + rows].
static hfe_status chain_ccmm_impl(const hfe_db* D, const hfe_qct* Qc, int64_t row0, int64_t rows, int32_t form,
                                  hipStream_t s, hfe_rct* R, Workspace& W, uint64_t* out_ext, uint64_t* C_ext) {
  const hfe_keys* K = D->keys;
  if (form != HFE_FORM_P2_I8) return fail(HFE_EINVAL, "the n^2 modulus chain runs HFE_FORM_P2_I8");
  const int level = Qc->level, np = K->cp, slots = np + level;
  int64_t d3 = Qc->d3, R_out = R->R_out;
  const int64_t ndb = 1ll << K->P.log_n_db;
  ChainLiftArgs la;
  std::memset(&la, 0, sizeof(la));
  la.level = level;
  la.np = np;
  uint64_t qm[HFE_MAX_QPRIMES];
  for (int j = 0; j < level; ++j) {
    qm[j] = K->cmod[j].q;
    la.q[j] = qm[j];
    la.mu[j] = K->cmod[j].mu;
    la.qmagic[j] = magic_u32((uint32_t)qm[j]);
  }
  garner_consts_of(qm, level, la.garner, la.half_digits);
  for (int t = 0; t < np; ++t) {
    const uint64_t pm = K->cmod[K->cq + t].q;
    la.pm[t] = pm;
    la.pmu[t] = K->cmod[K->cq + t].mu;
    la.pmagic[t] = magic_u32((uint32_t)pm);
    uint64_t prod = 1 % pm;
    for (int j = 0; j < level; ++j) {
      la.mprod[t][j] = prod;
      prod = mulmod(prod, qm[j] % pm, pm);
    }
    la.Q_mod[t] = prod;
    la.base[t] = chain_base(K->cbase[K->cq + t]);
  }
  for (int j = 0; j < level; ++j) la.base[np + j] = chain_base(K->cbase[j]);
  const int tq = p2_tile_q(&d3, &R_out, &slots, 1);
  const int64_t d3_pad = (d3 + tq - 1) / tq * tq;
  const size_t planeX = (size_t)D->KB * d3_pad * kKB;
  int8_t* Xd = nullptr;
  HFE_TRY(W.get((size_t)slots * 2 * planeX, s, &Xd));
  uint16_t* res = nullptr;
  HFE_TRY(W.get(sizeof(uint16_t) * (size_t)slots * d3 * R_out, s, &res));
  if (out_ext) {
    R->outp = out_ext;
  } else if (!C_ext) {
    HFE_TRY(R->out.alloc(sizeof(uint64_t) * (size_t)level * d3 * R_out, s));
    R->outp = R->out.as<uint64_t>();
  }
  const bool prof = g_profile.load() != 0 && W.base == nullptr && !C_ext;
  if (prof)
    for (auto& e : R->ev) HFE_LAUNCH(hipEventCreate(&e));
  auto mark = [&](int i) -> hipError_t { return prof ? hipEventRecord(R->ev[i], s) : hipSuccess; };
  HFE_LAUNCH(mark(0));
  HFE_LAUNCH(launch_chain_lift(Qc->XT.as<uint64_t>(), d3, D->K, D->KB, d3_pad, la, Xd, s));
  P2GemmArgs pg;
  std::memset(&pg, 0, sizeof(pg));
  pg.nz = 1;
  pg.n_bases = slots;
  pg.Dq[0] = D->p2.as<int8_t>();
  pg.Xq[0] = Xd;
  for (int j = 0; j < slots; ++j) {
    pg.n[j] = la.base[j].n;
    pg.m[j] = la.base[j].m;
    pg.rn[j] = la.base[j].rcp_n;
    pg.rm[j] = la.base[j].rcp_m;
  }
  pg.res = res;
  pg.KB = D->KB;
  pg.R_pad = D->R_pad;
  pg.n_db = ndb;
  pg.row0 = row0;
  pg.R_out = R_out;
  pg.d3 = d3;
  pg.d3_pad = d3_pad;
  HFE_LAUNCH(mark(1));
  HFE_LAUNCH(launch_gemm_p2(pg, tq, s));
  if (C_ext) return hip_ok_or_fail(launch_chain_widen(res, d3 * R_out, level, np, C_ext, s));
  HFE_LAUNCH(mark(2));
  ChainRescaleArgs ra;
  std::memset(&ra, 0, sizeof(ra));
  ra.level = level;
  ra.np = np;
  ra.P = K->cP;
  uint64_t pre = 1;
  for (int t = 0; t < np; ++t) {
    ra.pm[t] = la.pm[t];
    ra.pmu[t] = la.pmu[t];
    ra.pinv[t] = inv_mod(pre % la.pm[t], la.pm[t]);
    ra.pmagic[t] = la.pmagic[t];
    pre *= la.pm[t];
  }
  for (int j = 0; j < level; ++j) {
    ra.mod[j] = K->cmod[j];
    ra.Pinv[j] = inv_mod(K->cP % qm[j], qm[j]);
    ra.qmagic[j] = la.qmagic[j];
  }
  HFE_LAUNCH(launch_chain_rescale(res, d3 * R_out, ra, R->outp, s));
  HFE_LAUNCH(mark(3));
  return HFE_OK;
}

static hfe_status ccmm_impl(const hfe_db* D, const hfe_qct* Qc, int64_t row0, int64_t rows, int32_t form,
                            hipStream_t s, hfe_rct* R, uint64_t* C_ext = nullptr, Workspace* ws = nullptr,
                            uint64_t* out_ext = nullptr) {
  Workspace own;
  Workspace& W = ws ? *ws : own;
  const hfe_keys* K = D->keys;
  const int level = Qc->level;
  const int64_t ndb = 1ll << K->P.log_n_db;
  const int64_t d3 = Qc->d3;
  const int64_t R_out = ndb + rows;
  R->kind = kRct;
  R->stream = s;
  R->keys = K;
  R->level = level;
  R->d3 = d3;
  R->row0 = row0;
  R->rows = rows;
  R->R_out = R_out;
  if (K->family) return chain_ccmm_impl(D, Qc, row0, rows, form, s, R, W, out_ext, C_ext);

  const LiftArgs la = make_lift_args(K, level);
  const int nz = level + 1;
  auto slot = [&](int z) { return z < level ? z : K->L; };
  const bool prof = g_profile.load() != 0 && W.base == nullptr;  // no events in the allocation-free call
  if (prof)
    for (auto& e : R->ev) HFE_LAUNCH(hipEventCreate(&e));
  auto mark = [&](int i) -> hipError_t { return prof ? hipEventRecord(R->ev[i], s) : hipSuccess; };
  HFE_LAUNCH(mark(0));
  // the small-modulus forms reconstruct and rescale in one pass (no contraction output C)
  const bool fused = form == HFE_FORM_RNS_I8 || form == HFE_FORM_P2_I8;
  const bool product = C_ext != nullptr;
  uint64_t* Cp = C_ext;
  if (!fused && !product) HFE_TRY(W.get(sizeof(uint64_t) * (size_t)nz * d3 * R_out, s, &Cp));
  const RescaleArgs ra = make_rescale_args(K, level);
  if (out_ext) {
    R->outp = out_ext;
  } else if (!product) {
    HFE_TRY(R->out.alloc(sizeof(uint64_t) * (size_t)level * d3 * R_out, s));
    R->outp = R->out.as<uint64_t>();
  }
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nz = nz;
  g.K = D->K;
  g.KB = D->KB;
  g.R_db = D->R;
  g.R_pad = D->R_pad;
  g.n_db = ndb;
  g.row0 = row0;
  g.rows = rows;
  g.R_out = R_out;
  g.d3 = d3;
  g.d3_pad = (d3 + kQueryPad - 1) / kQueryPad * kQueryPad;
  for (int z = 0; z < nz; ++z) {
    g.C[z] = fused ? nullptr : Cp + (size_t)z * d3 * R_out;
    g.mod[z] = K->mods[slot(z)];
  }
  if (form == HFE_FORM_PLAIN_U64) {
    uint64_t* Xp = nullptr;
    HFE_TRY(W.get(sizeof(uint64_t) * (size_t)d3 * D->K, s, &Xp));
    HFE_LAUNCH(launch_lift(Qc->XT.as<uint64_t>(), d3, D->K, D->KB, g.d3_pad, la, Xp, nullptr, s));
    for (int z = 0; z < nz; ++z) {
      g.Dt[z] = D->Dt.as<uint64_t>() + (size_t)slot(z) * D->K * D->R;
      g.X[z] = z < level ? Qc->XT.as<uint64_t>() + (size_t)z * d3 * D->K : Xp;
    }
    HFE_LAUNCH(mark(1));
    HFE_LAUNCH(launch_gemm_plain(g, s));
  } else if (form == HFE_FORM_RNS_I8) {
    const int n = D->n_rns;
    const int tq = rns_tile_q(&d3, &R_out, &nz, 1);  // query tile width by padded work
    const int64_t d3_pad = (d3 + tq - 1) / tq * tq;   // whole query tiles
    const size_t planeX = (size_t)D->KB * d3_pad * kKB;
    const size_t planeD = (size_t)D->KB * D->R_pad * kKB;
    int8_t* Xd = nullptr;
    HFE_TRY(W.get((size_t)nz * n * planeX, s, &Xd));
    uint8_t* res = nullptr;
    HFE_TRY(W.get((size_t)nz * n * d3 * R_out, s, &res));
    HFE_LAUNCH(launch_lift_rns(Qc->XT.as<uint64_t>(), d3, D->K, D->KB, d3_pad, la, n, Xd, s));
    RnsGemmArgs rg;
    std::memset(&rg, 0, sizeof(rg));
    rg.nz = nz;
    rg.n_mod = n;
    for (int z = 0; z < nz; ++z) {
      rg.Dr[z] = D->rns.as<int8_t>() + (size_t)slot(z) * n * planeD;
      rg.Xr[z] = Xd + (size_t)z * n * planeX;
    }
    for (int j = 0; j < n; ++j) {
      rg.m[j] = kRnsMods[j];
      rg.magic[j] = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)kRnsMods[j] - 1) / (uint64_t)kRnsMods[j]);
    }
    rg.res = res;
    rg.KB = D->KB;
    rg.R_pad = D->R_pad;
    rg.n_db = ndb;
    rg.row0 = row0;
    rg.R_out = R_out;
    rg.d3 = d3;
    rg.d3_pad = d3_pad;
    HFE_LAUNCH(mark(1));
    HFE_LAUNCH(launch_gemm_rns(rg, tq, s));
    HFE_LAUNCH(mark(2));
    if (product)
      HFE_LAUNCH(launch_crt_rns(res, nz, d3 * R_out, make_rns_crt_args(K, level, n), Cp, s));
    else
      HFE_LAUNCH(launch_crt_rescale_rns(res, d3 * R_out, make_rns_crt_args(K, level, n), ra, R->outp, s));
  } else if (form == HFE_FORM_P2_I8) {
    const int n = D->n_p2;
    const int tq = p2_tile_q(&d3, &R_out, &nz, 1);  // query tile width by padded work
    const int64_t d3_pad = (d3 + tq - 1) / tq * tq;
    const size_t planeX = (size_t)D->KB * d3_pad * kKB;
    const size_t planeD = (size_t)D->KB * D->R_pad * kKB;
    int8_t* Xd = nullptr;
    HFE_TRY(W.get((size_t)nz * 2 * n * planeX, s, &Xd));
    uint16_t* res = nullptr;
    HFE_TRY(W.get(sizeof(uint16_t) * (size_t)nz * n * d3 * R_out, s, &res));
    HFE_LAUNCH(launch_lift_p2(Qc->XT.as<uint64_t>(), d3, D->K, D->KB, d3_pad, la, n, Xd, s));
    P2GemmArgs pg;
    std::memset(&pg, 0, sizeof(pg));
    pg.nz = nz;
    pg.n_bases = n;
    for (int z = 0; z < nz; ++z) {
      pg.Dq[z] = D->p2.as<int8_t>() + (size_t)slot(z) * 2 * n * planeD;
      pg.Xq[z] = Xd + (size_t)z * 2 * n * planeX;
    }
    for (int j = 0; j < n; ++j) {
      pg.n[j] = kP2Bases[j];
      pg.m[j] = kP2Bases[j] * kP2Bases[j];
      pg.rn[j] = 1.0 / (double)pg.n[j];
      pg.rm[j] = 1.0 / (double)pg.m[j];
    }
    pg.res = res;
    pg.KB = D->KB;
    pg.R_pad = D->R_pad;
    pg.n_db = ndb;
    pg.row0 = row0;
    pg.R_out = R_out;
    pg.d3 = d3;
    pg.d3_pad = d3_pad;
    HFE_LAUNCH(mark(1));
    HFE_LAUNCH(launch_gemm_p2(pg, tq, s));
    HFE_LAUNCH(mark(2));
    if (product)
      HFE_LAUNCH(launch_crt_p2(res, nz, d3 * R_out, make_p2_crt_args(K, level, n), Cp, s));
    else
      HFE_LAUNCH(launch_crt_rescale_p2(res, d3 * R_out, make_p2_crt_args(K, level, n), ra, R->outp, s));
  } else {
    const size_t planeX = (size_t)D->KB * g.d3_pad * kKB;
    const size_t planeD = (size_t)D->KB * D->R_pad * kKB;
    int8_t* Xd = nullptr;
    HFE_TRY(W.get((size_t)nz * kDigits * planeX, s, &Xd));
    HFE_LAUNCH(launch_lift(Qc->XT.as<uint64_t>(), d3, D->K, D->KB, g.d3_pad, la, nullptr, Xd, s));
    for (int z = 0; z < nz; ++z) {
      g.Dd[z] = D->digits.as<int8_t>() + (size_t)slot(z) * kDigits * planeD;
      g.Xd[z] = Xd + (size_t)z * kDigits * planeX;
    }
    HFE_LAUNCH(mark(1));
    HFE_LAUNCH(launch_gemm_i8(g, pick_i8_variant(level, d3), s));
  }
  if (!fused && !product) {
    HFE_LAUNCH(mark(2));
    HFE_LAUNCH(launch_rescale(Cp, Cp + (size_t)level * d3 * R_out, d3 * R_out, ra, R->outp, s));
  }
  HFE_LAUNCH(mark(3));
  return HFE_OK;
}

// Argument checks shared by the single-call CCMM entry points.
static hfe_status check_ccmm_args(const hfe_db* D, const hfe_qct* Qc, int64_t row0, int64_t rows, int32_t form) {
  if (!D || !Qc) return fail(HFE_EINVAL, "invalid database or query handle");
  if (Qc->keys != D->keys) return fail(HFE_EINVAL, "database and query use different keys");
  if (Qc->K != D->K) return fail(HFE_ESHAPE, "query and database code lengths differ");
  if (Qc->level > (D->keys->family ? D->keys->cq : D->keys->L))
    return fail(HFE_ELEVEL, "query level above the database primes");
  if (row0 < 0 || rows < 1 || row0 + rows > D->d1) return fail(HFE_ESHAPE, "row range outside the database");
  if (form != HFE_FORM_PLAIN_U64 && form != HFE_FORM_I8_MFMA && form != HFE_FORM_RNS_I8 && form != HFE_FORM_P2_I8)
    return fail(HFE_EINVAL, "unknown form");
  if (!(D->forms & (uint32_t)form)) return fail(HFE_EINVAL, "database not prepared for this form");
  return HFE_OK;
}

// The CCMM of hfe_ccmm with every device buffer of the call carved from [region, region + cap)
// and the rescaled result written to `out` ([level][d3][N_DB + rows]); nothing is allocated.
extern "C++" hfe_status hfe::ccmm_region(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                            hipStream_t s, uint64_t* out, void* region, size_t cap) {
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  const hfe_qct* Qc = as_handle<hfe_qct>(q, kQct);
  HFE_TRY(check_ccmm_args(D, Qc, row0, rows, form));
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  if (!region) return fail(HFE_EINTERNAL, "no scratch region");
  Workspace ws;
  ws.base = static_cast<uint8_t*>(region);
  ws.cap = cap;
  hfe_rct R;  // shape record only
  return ccmm_impl(D, Qc, row0, rows, form, s, &R, nullptr, &ws, out);
}

hfe_status hfe_ccmm(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form, void* stream,
                    hfe_rct** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  const hfe_qct* Qc = as_handle<hfe_qct>(q, kQct);
  HFE_TRY(check_ccmm_args(D, Qc, row0, rows, form));
  hfe_rct* R = new (std::nothrow) hfe_rct();
  if (!R) return fail(HFE_ENOMEM, "host allocation failed");
  hfe_status st = ccmm_impl(D, Qc, row0, rows, form, (hipStream_t)stream, R);
  if (st != HFE_OK) {
    delete R;
    return st;
  }
  *out = R;
  return HFE_OK;
}

hfe_status hfe_ccmm_product(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                            void* stream, uint64_t* C) {
  if (!C) return fail(HFE_EINVAL, "C is NULL");
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  const hfe_qct* Qc = as_handle<hfe_qct>(q, kQct);
  HFE_TRY(check_ccmm_args(D, Qc, row0, rows, form));
  hfe_rct R;  // shape record only; the buffers of the call are released in stream order on return
  return ccmm_impl(D, Qc, row0, rows, form, (hipStream_t)stream, &R, C);
}

hfe_status hfe_result_create(const hfe_db* db, const hfe_qct* q, void* stream, hfe_rct** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  const hfe_qct* Qc = as_handle<hfe_qct>(q, kQct);
  if (!D || !Qc) return fail(HFE_EINVAL, "invalid database or query handle");
  if (Qc->keys != D->keys) return fail(HFE_EINVAL, "database and query use different keys");
  hfe_rct* R = new (std::nothrow) hfe_rct();
  if (!R) return fail(HFE_ENOMEM, "host allocation failed");
  R->kind = kRct;
  R->stream = (hipStream_t)stream;
  R->keys = D->keys;
  R->level = Qc->level;
  R->d3 = Qc->d3;
  R->row0 = 0;
  R->rows = D->d1;
  R->R_out = (1ll << D->keys->P.log_n_db) + D->d1;
  hfe_status st = R->out.alloc(sizeof(uint64_t) * (size_t)R->level * R->d3 * R->R_out, (hipStream_t)stream);
  if (st != HFE_OK) {
    delete R;
    return st;
  }
  R->outp = R->out.as<uint64_t>();
  *out = R;
  return HFE_OK;
}

int32_t hfe_i8_variants(void) { return i8_variant_count(); }

const char* hfe_i8_variant_name(int32_t v) { return i8_variant_name(v); }

hfe_status hfe_set_i8_variant(int32_t v) {
  if (v < -1 || v >= i8_variant_count()) return fail(HFE_EINVAL, "no such i8 variant");
  g_i8_variant.store(v);
  return HFE_OK;
}

hfe_status hfe_profile(int32_t enable) {
  g_profile.store(enable ? 1 : 0);
  return HFE_OK;
}

hfe_status hfe_profile_ms(const hfe_rct* r, float* ms, int32_t n) {
  const hfe_rct* R = as_handle<hfe_rct>(r, kRct);
  if (!R || !ms || n < 0 || n > 3) return fail(HFE_EINVAL, "invalid result handle or count");
  if (!R->ev[0]) return fail(HFE_EINVAL, "result was produced without profiling");
  for (int i = 0; i < n; ++i) {
    HFE_LAUNCH(hipEventSynchronize(R->ev[i + 1]));
    HFE_LAUNCH(hipEventElapsedTime(&ms[i], R->ev[i], R->ev[i + 1]));
  }
  return HFE_OK;
}

// ------------------------------------------------------------------ batched CCMM
}  // extern "C"

FormShape hfe::form_shape(const hfe_db* D, int form) {
  FormShape f;
  f.rns = form == HFE_FORM_RNS_I8;
  f.p2 = form == HFE_FORM_P2_I8;
  f.planes = f.rns ? D->n_rns : f.p2 ? 2 * D->n_p2 : kDigits;
  f.qpad = f.rns ? kRnsTileQ : f.p2 ? kP2TileQ : kQueryPad;
  f.res_bytes = f.rns ? 1 : f.p2 ? 2 : 0;
  f.lift_form = f.rns ? D->n_rns : f.p2 ? -D->n_p2 : 0;
  return f;
}

namespace {
// Byte layout of the descriptor tables of a batch of up to `items` items and `problems` problems
// (256-byte aligned parts): contraction (per problem), lift (per item), rescale (per item), RNS
// reconstruction (per problem).
struct BlobLayout {
  size_t gh, gd, lh, ld, rh, rd, ch, cd, bytes;
  BlobLayout(int items, int problems) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    gh = 0;
    gd = al(gh + sizeof(BatchHeader));
    lh = al(gd + sizeof(BatchDesc) * problems);
    ld = al(lh + sizeof(BatchElemHeader));
    rh = al(ld + sizeof(BatchLiftDesc) * items);
    rd = al(rh + sizeof(BatchElemHeader));
    ch = al(rd + sizeof(BatchRescaleDesc) * items);
    cd = al(ch + sizeof(BatchElemHeader));
    bytes = al(cd + sizeof(BatchCrtDesc) * problems);
  }
};
// problems of a batch of n items: at most one more per level than items (see group_items)
int max_problems(int n) { return n + kMaxPrimes; }

struct BatchSizes {
  size_t xd_bytes = 0, c_elems = 0, res_bytes = 0, out_elems = 0;
  int64_t cols = 0;
  int max_level = 0, problems = 0;
};

hfe_status check_item(const hfe_db* D, const hfe_batch_item& it) {
  const hfe_qct* Qc = as_handle<hfe_qct>(it.q, kQct);
  if (!Qc) return fail(HFE_EINVAL, "invalid query handle in batch");
  if (Qc->keys != D->keys) return fail(HFE_EINVAL, "database and query use different keys");
  if (Qc->K != D->K) return fail(HFE_ESHAPE, "query and database code lengths differ");
  if (Qc->level > D->keys->L) return fail(HFE_ELEVEL, "query level above the database primes");
  if (it.row0 < 0 || it.rows < 1 || it.row0 + it.rows > D->d1) return fail(HFE_ESHAPE, "row range outside the database");
  return HFE_OK;
}

// Problems of a batch.  Every item multiplies the database's N_DB A rows and its own range of B
// rows.  The items of one level that share a row range form one problem (A rows and that range,
// their query columns side by side).  A level whose items cover several row ranges is split:
// one problem over the A rows for all of the level's columns, padded to whole tiles once, and one
// problem per row range over just its B rows, which reads its columns from the A problem's query
// planes (the level's columns are ordered by row range there, so each range's columns are
// contiguous).  Every item's query planes are lifted once, into its owner problem.
struct Problem {
  int level = 0;
  int64_t row0 = 0, rows = 0;  // B rows of the problem (rows = 0: A rows only)
  bool a_rows = true;          // the problem includes the A rows
  int64_t d3 = 0;              // query columns
  int owner = 0;               // problem holding these columns' query planes (itself, or its A problem)
  int64_t xc0 = 0;             // first column in the owner's planes
  int last_item = -1;          // owners: the item whose columns come last (it also fills the padding)
};
struct Grouping {
  std::vector<Problem> p;
  std::vector<int> pa, pb;      // per item: problem of its A rows, of its B rows
  std::vector<int64_t> ca, cb;  // per item: first column in those problems
};

Grouping group_items(const hfe_batch_item* items, int n) {
  Grouping g;
  g.pa.resize(n);
  g.pb.resize(n);
  g.ca.resize(n);
  g.cb.resize(n);
  auto level_of = [&](int i) { return static_cast<const hfe_qct*>(items[i].q)->level; };
  auto d3_of = [&](int i) { return static_cast<const hfe_qct*>(items[i].q)->d3; };
  std::vector<int> levels;                       // in order of first appearance
  std::vector<std::vector<std::vector<int>>> by;  // per level: per row range (first appearance): items
  for (int i = 0; i < n; ++i) {
    size_t l = 0;
    while (l < levels.size() && levels[l] != level_of(i)) ++l;
    if (l == levels.size()) {
      levels.push_back(level_of(i));
      by.emplace_back();
    }
    size_t r = 0;
    while (r < by[l].size() &&
           !(items[by[l][r][0]].row0 == items[i].row0 && items[by[l][r][0]].rows == items[i].rows))
      ++r;
    if (r == by[l].size()) by[l].emplace_back();
    by[l][r].push_back(i);
  }
  for (size_t l = 0; l < levels.size(); ++l) {
    const int A = (int)g.p.size();
    Problem pa;
    pa.level = levels[l];
    pa.owner = A;
    if (by[l].size() == 1) {  // one row range: one problem
      pa.row0 = items[by[l][0][0]].row0;
      pa.rows = items[by[l][0][0]].rows;
    }
    g.p.push_back(pa);
    for (const auto& range : by[l]) {
      int B = A;
      if (by[l].size() > 1) {
        B = (int)g.p.size();
        Problem pb;
        pb.level = levels[l];
        pb.row0 = items[range[0]].row0;
        pb.rows = items[range[0]].rows;
        pb.a_rows = false;
        pb.owner = A;
        pb.xc0 = g.p[A].d3;
        g.p.push_back(pb);
      }
      for (int i : range) {
        g.pa[i] = A;
        g.ca[i] = g.p[A].d3;
        g.p[A].d3 += d3_of(i);
        g.p[A].last_item = i;
        g.pb[i] = B;
        if (B != A) {
          g.cb[i] = g.p[B].d3;
          g.p[B].d3 += d3_of(i);
        } else {
          g.cb[i] = g.ca[i];
        }
      }
    }
  }
  return g;
}

// Sizes of a batch for a form (HFE_FORM_I8_MFMA with the digit tile `variant`, HFE_FORM_RNS_I8 or
// HFE_FORM_P2_I8),
// and (when blob != nullptr) its descriptor tables pointing into the given workspace (xd_base,
// c_base, res_base) and result arrays (outs[i]).
BatchSizes batch_fill(const hfe_db* D, const hfe_batch_item* items, int n, int form, int variant, int8_t* xd_base,
                      uint64_t* c_base, uint8_t* res_base, uint64_t* const* outs, uint8_t* blob,
                      const BlobLayout& L) {
  const hfe_keys* K = D->keys;
  const int64_t ndb = 1ll << K->P.log_n_db;
  const FormShape fs = form_shape(D, form);
  const bool rns = fs.rns, small = fs.res_bytes > 0;
  const int planes = fs.planes;
  const int64_t qpad = fs.qpad;
  const Grouping gr = group_items(items, n);
  const int np = (int)gr.p.size();
  BatchSizes z;
  z.problems = np;
  std::vector<size_t> xd_off(np), c_off(np), res_off(np);
  std::vector<int64_t> d3_pad(np), R_out(np);
  std::vector<char> feeds(np, 0);  // owners whose planes split problems also read
  for (int b = 0; b < np; ++b)
    if (gr.p[b].owner != b) feeds[gr.p[b].owner] = 1;
  for (int b = 0; b < np; ++b) R_out[b] = (gr.p[b].a_rows ? ndb : 0) + gr.p[b].rows;
  // RNS and n^2 forms: each problem's query tile width by its own padded work; the 256-column problems come
  // first in the tables (one launch each width).  Owners' planes are padded for the widest tiles.
  std::vector<int> tq(np, 0), ord(np);
  for (int b = 0; b < np; ++b) {
    ord[b] = b;
    const int nzb = gr.p[b].level + 1;
    if (rns) tq[b] = rns_tile_q(&gr.p[b].d3, &R_out[b], &nzb, 1);
    if (fs.p2) tq[b] = p2_tile_q(&gr.p[b].d3, &R_out[b], &nzb, 1);
  }
  if (small) std::stable_partition(ord.begin(), ord.end(), [&](int b) { return tq[b] == 256; });
  // query planes of the owners: whole tiles, and for an owner that feeds split problems room for
  // their last tile, which may reach qpad - 1 columns past the owner's columns
  for (int b = 0; b < np; ++b) {
    const Problem& P = gr.p[b];
    if (P.owner != b) continue;
    d3_pad[b] = (P.d3 + (feeds[b] ? qpad - 1 : 0) + qpad - 1) / qpad * qpad;
    xd_off[b] = z.xd_bytes;
    z.xd_bytes += (size_t)(P.level + 1) * planes * D->KB * d3_pad[b] * kKB;
  }
  int64_t tiles = 0, crt_e = 0, tiles_wide = 0;
  int n_wide = 0;
  for (int k = 0; k < np; ++k) {
    const int b = ord[k];  // table position k
    const Problem& P = gr.p[b];
    const int level = P.level, nz = level + 1;
    const int64_t d3 = P.d3;
    c_off[b] = z.c_elems;
    res_off[b] = z.res_bytes;
    if (blob) {
      BatchDesc& g = reinterpret_cast<BatchDesc*>(blob + L.gd)[k];
      std::memset(&g, 0, sizeof(g));
      g.Xd = xd_base + xd_off[P.owner] + P.xc0 * kKB;
      g.C = c_base + c_off[b];
      g.res = small ? res_base + res_off[b] : nullptr;
      // output row r < n_db is database row r, row r >= n_db is row n_db + row0 + (r - n_db)
      g.n_db = P.a_rows ? ndb : 0;
      g.row0 = P.a_rows ? P.row0 : ndb + P.row0;
      g.R_out = R_out[b];
      g.d3 = d3;
      g.d3_pad = d3_pad[P.owner];
      g.tile_begin = tiles;
      g.nz = nz;
      for (int zz = 0; zz < nz; ++zz) {
        g.slot[zz] = zz < level ? zz : K->L;
        g.mod[zz] = K->mods[g.slot[zz]];
      }
      if (small) {
        BatchCrtDesc& c = reinterpret_cast<BatchCrtDesc*>(blob + L.cd)[k];
        std::memset(&c, 0, sizeof(c));
        c.res = g.res;
        c.C = g.C;
        c.n = d3 * R_out[b];
        c.elem_begin = crt_e;
        c.nz = nz;
        c.level = level;
        c.pslot = K->L;
      }
    }
    tiles += rns      ? rns_batched_tiles(d3, R_out[b], nz, planes, tq[b])
             : fs.p2 ? p2_batched_tiles(d3, R_out[b], nz, D->n_p2, tq[b])
                     : i8_batched_tiles(variant, d3, R_out[b], nz);
    if (small && tq[b] == 256) {
      tiles_wide = tiles;
      n_wide = k + 1;
    }
    // the CRT's unit: 4 entries (RNS form) or 2 (n^2 form) of one prime slot
    const int64_t unit = fs.p2 ? 2 : 4;
    crt_e += ((int64_t)nz * ((d3 * R_out[b] + unit - 1) / unit) + 255) / 256 * 256;
    // each problem's C starts at a multiple of 4 entries and its residues at a multiple of 8 bytes
    // (the CRT's word loads and 16-byte stores)
    z.c_elems += ((size_t)nz * d3 * R_out[b] + 3) / 4 * 4;
    if (small) z.res_bytes += ((size_t)nz * (fs.p2 ? D->n_p2 : planes) * d3 * R_out[b] * fs.res_bytes + 7) / 8 * 8;
    z.max_level = std::max(z.max_level, level);
  }
  int64_t lift_e = 0, resc_e = 0;
  for (int i = 0; i < n; ++i) {
    const hfe_qct* Qc = static_cast<const hfe_qct*>(items[i].q);
    const int level = Qc->level;
    const int64_t d3 = Qc->d3;
    const int a = gr.pa[i], bb = gr.pb[i];  // the A problem is the owner of the item's planes
    const int64_t R_item = ndb + items[i].rows;
    // the owner's last item also writes the padding columns (zeros)
    const int64_t cols = d3 + (gr.p[a].last_item == i ? d3_pad[a] - (gr.ca[i] + d3) : 0);
    if (blob) {
      BatchLiftDesc& l = reinterpret_cast<BatchLiftDesc*>(blob + L.ld)[i];
      std::memset(&l, 0, sizeof(l));
      l.XT = Qc->XT.as<uint64_t>();
      l.Xd = xd_base + xd_off[a];
      l.d3 = d3;
      l.c0 = gr.ca[i];
      l.cols = cols;
      l.d3_pad = d3_pad[a];
      l.elem_begin = lift_e;
      l.la = make_lift_args(K, level);
      BatchRescaleDesc& r = reinterpret_cast<BatchRescaleDesc*>(blob + L.rd)[i];
      std::memset(&r, 0, sizeof(r));
      r.C = c_base + c_off[a] + gr.ca[i] * R_out[a];
      r.Ra = R_out[a];
      r.zstride = gr.p[a].d3 * R_out[a];
      if (bb == a) {  // every row in the one problem
        r.Cb = r.C;
        r.Rb = r.Ra;
        r.zstride_b = r.zstride;
        r.split = R_item;
      } else {
        r.Cb = c_base + c_off[bb] + gr.cb[i] * R_out[bb];
        r.Rb = R_out[bb];
        r.zstride_b = gr.p[bb].d3 * R_out[bb];
        r.split = ndb;
      }
      r.R_out = R_item;
      r.out = outs[i];
      r.n = d3 * R_item;
      r.elem_begin = resc_e;
      r.ra = make_rescale_args(K, level);
    }
    lift_e += (cols * D->KB * kKB + 255) / 256 * 256;
    resc_e += (d3 * R_item + 255) / 256 * 256;
    z.out_elems += (size_t)level * d3 * R_item;
    z.cols += d3;
  }
  if (blob) {
    BatchHeader* gh = reinterpret_cast<BatchHeader*>(blob + L.gh);
    gh->total_tiles = tiles;
    gh->n = np;
    gh->tiles_wide = small ? tiles_wide : tiles;
    gh->n_wide = small ? n_wide : np;
    BatchElemHeader* lh = reinterpret_cast<BatchElemHeader*>(blob + L.lh);
    lh->total = lift_e;
    lh->n = n;
    BatchElemHeader* rh = reinterpret_cast<BatchElemHeader*>(blob + L.rh);
    rh->total = resc_e;
    rh->n = n;
    BatchElemHeader* ch = reinterpret_cast<BatchElemHeader*>(blob + L.ch);
    ch->total = small ? crt_e : 0;
    ch->n = small ? np : 0;
  }
  return z;
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    else
      cus = 256;
  }
  return cus;
}

int gemm_grid_for(int form, int variant) {
  // RNS form: variant is the query tile width (256 or 128); n^2 form: one workgroup per CU
  const int g = device_cus() * (form == HFE_FORM_RNS_I8  ? rns_wgs_per_cu(variant)
                                : form == HFE_FORM_P2_I8 ? 1
                                                         : i8_variant_wgs_per_cu(variant));
  return (g + kXcds - 1) / kXcds * kXcds;
}
constexpr int kElemGrid = 4096;

hfe_status batch_enqueue(const hfe_db* D, const uint8_t* dblob, const BlobLayout& L, int form, int variant,
                         int elem_grid, hipStream_t s) {
  const bool rns = form == HFE_FORM_RNS_I8;
  HFE_LAUNCH(launch_lift_batched(reinterpret_cast<const BatchElemHeader*>(dblob + L.lh),
                                 reinterpret_cast<const BatchLiftDesc*>(dblob + L.ld), D->K, D->KB,
                                 form_shape(D, form).lift_form, elem_grid, s));
  const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(dblob + L.gh);
  if (rns) {
    RnsBatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.hdr = hdr;
    a.next = const_cast<uint32_t*>(hdr->next);
    a.next_narrow = const_cast<uint32_t*>(hdr->next_narrow);
    a.desc = reinterpret_cast<const BatchDesc*>(dblob + L.gd);
    a.Dr = D->rns.as<int8_t>();
    a.n_mod = D->n_rns;
    for (int j = 0; j < D->n_rns; ++j) {
      a.m[j] = kRnsMods[j];
      a.magic[j] = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)kRnsMods[j] - 1) / (uint64_t)kRnsMods[j]);
    }
    a.KB = D->KB;
    a.R_pad = D->R_pad;
    // the 256-column problems, then the 128-column ones (either launch may find no tiles)
    HFE_LAUNCH(launch_gemm_rns_batched(a, gemm_grid_for(form, 256), 256, s));
    HFE_LAUNCH(launch_gemm_rns_batched(a, gemm_grid_for(form, 128), 128, s));
    // by-slot constants: level L makes z index the database slot
    HFE_LAUNCH(launch_crt_rns_batched(reinterpret_cast<const BatchElemHeader*>(dblob + L.ch),
                                      reinterpret_cast<const BatchCrtDesc*>(dblob + L.cd),
                                      make_rns_crt_args(D->keys, D->keys->L, D->n_rns), elem_grid, s));
  } else if (form == HFE_FORM_P2_I8) {
    P2BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.hdr = hdr;
    a.next = const_cast<uint32_t*>(hdr->next);
    a.next_narrow = const_cast<uint32_t*>(hdr->next_narrow);
    a.desc = reinterpret_cast<const BatchDesc*>(dblob + L.gd);
    a.Dq = D->p2.as<int8_t>();
    a.n_bases = D->n_p2;
    a.KB = D->KB;
    a.R_pad = D->R_pad;
    // the 256-column problems, then the 128-column ones (either launch may find no tiles)
    HFE_LAUNCH(launch_gemm_p2_batched(a, gemm_grid_for(form, 0), 256, s));
    HFE_LAUNCH(launch_gemm_p2_batched(a, gemm_grid_for(form, 0), 128, s));
    HFE_LAUNCH(launch_crt_p2_batched(reinterpret_cast<const BatchElemHeader*>(dblob + L.ch),
                                     reinterpret_cast<const BatchCrtDesc*>(dblob + L.cd),
                                     make_p2_crt_args(D->keys, D->keys->L, D->n_p2), elem_grid, s));
  } else {
    BatchGemmArgs a;
    a.hdr = hdr;
    a.next = const_cast<uint32_t*>(hdr->next);
    a.desc = reinterpret_cast<const BatchDesc*>(dblob + L.gd);
    a.Dd = D->digits.as<int8_t>();
    a.KB = D->KB;
    a.R_pad = D->R_pad;
    HFE_LAUNCH(launch_gemm_i8_batched(a, variant, gemm_grid_for(form, variant), s));
  }
  HFE_LAUNCH(launch_rescale_batched(reinterpret_cast<const BatchElemHeader*>(dblob + L.rh),
                                    reinterpret_cast<const BatchRescaleDesc*>(dblob + L.rd), elem_grid, s));
  return HFE_OK;
}

// Digit tile configuration of a batch: the forced one if set; else, of the configuration tuned for
// the batch's largest level and mean column count and the default one, the one whose tiles pad the
// batch's problems least (MFMA work including padded rows and columns); ties go to the tuned one.
int choose_batch_variant(const hfe_db* D, const hfe_batch_item* items, int n, int max_level, int64_t mean_cols) {
  if (g_i8_variant.load() >= 0) return g_i8_variant.load();
  const int tuned = pick_i8_variant(max_level, mean_cols);
  if (tuned == kDefaultI8Variant) return tuned;
  const int64_t ndb = 1ll << D->keys->P.log_n_db;
  const Grouping gr = group_items(items, n);
  auto padded = [&](int v) {
    const int64_t br = i8_variant_tile_rows(v), bq = i8_variant_tile_cols(v);
    double w = 0;
    for (const Problem& P : gr.p) {
      const int64_t R = (P.a_rows ? ndb : 0) + P.rows;
      w += (double)(P.level + 1) * ((P.d3 + bq - 1) / bq * bq) * ((R + br - 1) / br * br);
    }
    return w;
  };
  return padded(kDefaultI8Variant) < padded(tuned) ? kDefaultI8Variant : tuned;
}

}  // namespace

extern "C" {

hfe_status hfe_ccmm_batched(const hfe_db* db, const hfe_batch_item* items, int32_t n, int32_t form, void* stream,
                            hfe_rct** outs) {
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  if (!D || !items || !outs) return fail(HFE_EINVAL, "invalid database, items or outs");
  if (D->keys->family) return fail(HFE_EINVAL, "batches do not run the n^2 modulus chain");
  if (n < 1 || n > kMaxBatch) return fail(HFE_EINVAL, "batch size must be 1 .. 256");
  if (form != HFE_FORM_PLAIN_U64 && form != HFE_FORM_I8_MFMA && form != HFE_FORM_RNS_I8 && form != HFE_FORM_P2_I8)
    return fail(HFE_EINVAL, "unknown form");
  if (!(D->forms & (uint32_t)form)) return fail(HFE_EINVAL, "database not prepared for this form");
  for (int i = 0; i < n; ++i) {
    outs[i] = nullptr;
    HFE_TRY(check_item(D, items[i]));
  }
  hipStream_t s = (hipStream_t)stream;
  if (form == HFE_FORM_PLAIN_U64) {  // one call per item
    for (int i = 0; i < n; ++i) {
      hfe_status st = hfe_ccmm(db, items[i].q, items[i].row0, items[i].rows, form, stream, &outs[i]);
      if (st != HFE_OK) {
        for (int j = 0; j < i; ++j) hfe_free(outs[j]);
        return st;
      }
    }
    return HFE_OK;
  }
  // all problems of one batch use one tile configuration
  const BlobLayout L(n, max_problems(n));
  const BatchSizes sz0 = batch_fill(D, items, n, form, 0, nullptr, nullptr, nullptr, nullptr, nullptr, L);
  const int variant = form == HFE_FORM_I8_MFMA ? choose_batch_variant(D, items, n, sz0.max_level, sz0.cols / n) : 0;
  const hfe_keys* K = D->keys;
  const int64_t ndb = 1ll << K->P.log_n_db;
  std::vector<hfe_rct*> R(n, nullptr);
  auto cleanup = [&]() {
    for (auto* r : R) delete r;
  };
  std::vector<uint64_t*> outp(n);
  for (int i = 0; i < n; ++i) {
    const hfe_qct* Qc = static_cast<const hfe_qct*>(items[i].q);
    hfe_rct* r = new (std::nothrow) hfe_rct();
    if (!r) {
      cleanup();
      return fail(HFE_ENOMEM, "host allocation failed");
    }
    R[i] = r;
    r->kind = kRct;
    r->stream = s;
    r->keys = K;
    r->level = Qc->level;
    r->d3 = Qc->d3;
    r->row0 = items[i].row0;
    r->rows = items[i].rows;
    r->R_out = ndb + items[i].rows;
    hfe_status st = r->out.alloc(sizeof(uint64_t) * (size_t)r->level * r->d3 * r->R_out, s);
    if (st != HFE_OK) {
      cleanup();
      return st;
    }
    r->outp = r->out.as<uint64_t>();
    outp[i] = r->outp;
  }
  DevBuf Xd, C, res, blob;
  hfe_status st = Xd.alloc(sz0.xd_bytes, s);
  if (st == HFE_OK) st = C.alloc(sizeof(uint64_t) * sz0.c_elems, s);
  if (st == HFE_OK && sz0.res_bytes) st = res.alloc(sz0.res_bytes, s);
  if (st == HFE_OK) st = blob.alloc(L.bytes, s);
  if (st != HFE_OK) {
    cleanup();
    return st;
  }
  std::vector<uint8_t> host(L.bytes, 0);
  batch_fill(D, items, n, form, variant, Xd.as<int8_t>(), C.as<uint64_t>(), res.as<uint8_t>(), outp.data(),
             host.data(), L);
  hipError_t e = hipMemcpyAsync(blob.ptr, host.data(), L.bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the pageable staging is freed on return
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "descriptor upload");
  }
  st = batch_enqueue(D, blob.as<uint8_t>(), L, form, variant, kElemGrid, s);
  if (st != HFE_OK) {
    cleanup();
    return st;
  }
  for (int i = 0; i < n; ++i) outs[i] = R[i];
  return HFE_OK;
}

// A plan with the given workspace capacities (bytes of query planes and small-modulus residues,
// elements of the contraction output and of the results).
static hfe_status plan_alloc(const hfe_db* D, int form, int32_t max_items, int64_t max_cols, int max_level,
                             size_t xd_cap, size_t c_cap, size_t res_cap, size_t out_cap, hfe_plan** out) {
  hfe_plan* P = new (std::nothrow) hfe_plan();
  if (!P) return fail(HFE_ENOMEM, "host allocation failed");
  P->kind = kPlan;
  P->stream = nullptr;
  P->db = D;
  P->form = form;
  P->max_items = max_items;
  P->max_cols = max_cols;
  P->max_level = max_level;
  P->xd_cap = xd_cap;
  P->c_cap = c_cap;
  P->res_cap = res_cap;
  P->out_cap = out_cap;
  const BlobLayout L(max_items, max_problems(max_items));
  P->blob_bytes = L.bytes;
  hfe_status st = P->ws_xd.alloc(P->xd_cap, nullptr);
  if (st == HFE_OK) st = P->ws_c.alloc(sizeof(uint64_t) * P->c_cap, nullptr);
  if (st == HFE_OK && P->res_cap) st = P->ws_res.alloc(P->res_cap, nullptr);
  if (st == HFE_OK) st = P->ws_out.alloc(sizeof(uint64_t) * P->out_cap, nullptr);
  if (st == HFE_OK) st = P->desc.alloc(L.bytes, nullptr);
  hipError_t e = hipSuccess;
  if (st == HFE_OK) e = hipHostMalloc(&P->host_blob, L.bytes, hipHostMallocDefault);
  if (st == HFE_OK && e == hipSuccess) e = hipEventCreateWithFlags(&P->copied, hipEventDisableTiming);
  if (st == HFE_OK && e != hipSuccess) st = hip_fail(e, "plan staging");
  if (st != HFE_OK) {
    delete P;
    return st;
  }
  P->elem_grid = kElemGrid;
  for (int i = 0; i < max_items; ++i) {
    hfe_rct* v = new (std::nothrow) hfe_rct();
    if (!v) {
      delete P;
      return fail(HFE_ENOMEM, "host allocation failed");
    }
    v->kind = kRct;
    v->is_view = true;
    v->keys = D->keys;
    P->views.push_back(v);
  }
  *out = P;
  return HFE_OK;
}

static hfe_status check_plan_form(const hfe_db* D, int32_t form) {
  if (!D) return fail(HFE_EINVAL, "invalid database handle");
  if (D->keys->family) return fail(HFE_EINVAL, "plans do not run the n^2 modulus chain");
  if (form != HFE_FORM_I8_MFMA && form != HFE_FORM_RNS_I8 && form != HFE_FORM_P2_I8)
    return fail(HFE_EINVAL, "plans run an int8 form");
  if (!(D->forms & (uint32_t)form)) return fail(HFE_EINVAL, "database not prepared for this form");
  return HFE_OK;
}

hfe_status hfe_plan_create(const hfe_db* db, int32_t max_items, int64_t max_cols, uint32_t max_level, int32_t form,
                           hfe_plan** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  HFE_TRY(check_plan_form(D, form));
  if (max_items < 1 || max_items > kMaxBatch) return fail(HFE_EINVAL, "max_items must be 1 .. 256");
  if (max_cols < 1 || max_level < 1 || (int)max_level > D->keys->L) return fail(HFE_EINVAL, "bad capacity");
  const FormShape fs = form_shape(D, form);
  const int planes = fs.planes;
  const int64_t qpad = fs.qpad;
  const int64_t ndb = 1ll << D->keys->P.log_n_db;
  const int64_t R_max = ndb + D->d1;
  // an owner problem pads at most qpad - 1 columns per item (two items at least when it also feeds
  // split problems, which need up to 2 (qpad - 1))
  const int64_t cols_pad = max_cols + (int64_t)max_items * (qpad - 1);
  const size_t xd_cap = (size_t)(max_level + 1) * planes * D->KB * cols_pad * kKB;
  // + the alignment of each problem's start
  const size_t c_cap = (size_t)(max_level + 1) * max_cols * R_max + 4 * (size_t)max_problems(max_items);
  // residues of the small-modulus forms (bytes; one per modulus or two per base), each problem's
  // start aligned to 8 bytes
  const int res_planes = fs.p2 ? D->n_p2 : fs.rns ? D->n_rns : 0;
  const size_t res_cap = fs.res_bytes ? (size_t)(max_level + 1) * res_planes * max_cols * R_max * fs.res_bytes +
                                            8 * (size_t)max_problems(max_items)
                                      : 0;
  const size_t out_cap = (size_t)max_level * max_cols * R_max;
  return plan_alloc(D, form, max_items, max_cols, (int)max_level, xd_cap, c_cap, res_cap, out_cap, out);
}

hfe_status hfe_plan_create_for(const hfe_db* db, const hfe_batch_item* items, int32_t n, int32_t form,
                               hfe_plan** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const hfe_db* D = as_handle<hfe_db>(db, kDb);
  HFE_TRY(check_plan_form(D, form));
  if (!items || n < 1 || n > kMaxBatch) return fail(HFE_EINVAL, "a batch holds 1 .. 256 items");
  for (int i = 0; i < n; ++i) HFE_TRY(check_item(D, items[i]));
  const BlobLayout L(n, max_problems(n));
  const BatchSizes sz = batch_fill(D, items, n, form, 0, nullptr, nullptr, nullptr, nullptr, nullptr, L);
  return plan_alloc(D, form, n, sz.cols, sz.max_level, sz.xd_bytes, sz.c_elems, sz.res_bytes, sz.out_elems, out);
}

hfe_status hfe_plan_run(hfe_plan* plan, const hfe_batch_item* items, int32_t n, int32_t use_graph, void* stream) {
  hfe_plan* P = as_handle<hfe_plan>(plan, kPlan);
  if (!P || !items) return fail(HFE_EINVAL, "invalid plan or items");
  if (n < 1 || n > P->max_items) return fail(HFE_EINVAL, "batch larger than the plan");
  const hfe_db* D = P->db;
  for (int i = 0; i < n; ++i) {
    HFE_TRY(check_item(D, items[i]));
    if (static_cast<const hfe_qct*>(items[i].q)->level > P->max_level)
      return fail(HFE_ELEVEL, "item level above the plan's maximum");
  }
  const BlobLayout L(P->max_items, max_problems(P->max_items));
  const BatchSizes sz = batch_fill(D, items, n, P->form, 0, nullptr, nullptr, nullptr, nullptr, nullptr, L);
  const int variant =
      P->form == HFE_FORM_I8_MFMA ? choose_batch_variant(D, items, n, sz.max_level, sz.cols / n) : 0;
  if (sz.cols > P->max_cols || sz.xd_bytes > P->xd_cap || sz.c_elems > P->c_cap || sz.res_bytes > P->res_cap ||
      sz.out_elems > P->out_cap)
    return fail(HFE_ESHAPE, "batch exceeds the plan's workspace");
  hipStream_t s = (hipStream_t)stream;
  // result views: consecutive slices of the output workspace
  const int64_t ndb = 1ll << D->keys->P.log_n_db;
  std::vector<uint64_t*> outp(n);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const hfe_qct* Qc = static_cast<const hfe_qct*>(items[i].q);
    hfe_rct* v = P->views[i];
    v->stream = s;
    v->level = Qc->level;
    v->d3 = Qc->d3;
    v->row0 = items[i].row0;
    v->rows = items[i].rows;
    v->R_out = ndb + items[i].rows;
    v->outp = P->ws_out.as<uint64_t>() + off;
    outp[i] = v->outp;
    off += (size_t)v->level * v->d3 * v->R_out;
  }
  // the pinned staging may still feed the previous run's upload
  HFE_LAUNCH(hipEventSynchronize(P->copied));
  uint8_t* host = static_cast<uint8_t*>(P->host_blob);
  std::memset(host, 0, P->blob_bytes);
  batch_fill(D, items, n, P->form, variant, P->ws_xd.as<int8_t>(), P->ws_c.as<uint64_t>(),
             P->ws_res.as<uint8_t>(), outp.data(), host, L);
  HFE_LAUNCH(hipMemcpyAsync(P->desc.ptr, host, P->blob_bytes, hipMemcpyHostToDevice, s));
  HFE_LAUNCH(hipEventRecord(P->copied, s));
  if (!use_graph) {
    HFE_TRY(batch_enqueue(D, P->desc.as<uint8_t>(), L, P->form, variant, P->elem_grid, s));
  } else {
    if (!P->exec[variant]) {
      // capture on a private stream that joins the caller's stream through events
      hipStream_t cap;
      HFE_LAUNCH(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hfe_status st = HFE_OK;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) st = batch_enqueue(D, P->desc.as<uint8_t>(), L, P->form, variant, P->elem_grid, cap);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(cap, &g);
      (void)hipStreamDestroy(cap);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e != hipSuccess ? e : e2, "graph capture");
      }
      if (st != HFE_OK) {
        (void)hipGraphDestroy(g);
        return st;
      }
      P->graph[variant] = g;
      HFE_LAUNCH(hipGraphInstantiate(&P->exec[variant], g, nullptr, nullptr, 0));
    }
    HFE_LAUNCH(hipGraphLaunch(P->exec[variant], s));
  }
  P->n_last = n;
  return HFE_OK;
}

hfe_status hfe_plan_result(const hfe_plan* plan, int32_t i, const hfe_rct** view) {
  const hfe_plan* P = as_handle<hfe_plan>(plan, kPlan);
  if (!P || !view) return fail(HFE_EINVAL, "invalid plan or view");
  if (i < 0 || i >= P->n_last) return fail(HFE_EINVAL, "no such item in the last run");
  *view = P->views[i];
  return HFE_OK;
}

// ------------------------------------------------------------------ autotuner
hfe_status hfe_autotune(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t reps, void* stream,
                        int32_t* best) {
  const hfe_qct* Qc = as_handle<hfe_qct>(q, kQct);
  if (!Qc || !best || reps < 1) return fail(HFE_EINVAL, "invalid query, best or reps");
  const int saved_variant = g_i8_variant.load();
  const int saved_profile = g_profile.load();
  // one untimed run per configuration, then `reps` rounds that time every configuration once each
  // (interleaved, so a drift of the clock over the tuning run favours none), keeping each one's best
  const int nv = i8_variant_count();
  std::vector<float> vbest(nv, 1e30f);
  hfe_status st = HFE_OK;
  for (int r = 0; r <= reps && st == HFE_OK; ++r) {
    for (int v = 0; v < nv && st == HFE_OK; ++v) {
      g_i8_variant.store(v);
      g_profile.store(r > 0 ? 1 : 0);
      hfe_rct* res = nullptr;
      st = hfe_ccmm(db, q, row0, rows, HFE_FORM_I8_MFMA, stream, &res);
      if (st == HFE_OK && r > 0) {
        float ms[2];
        st = hfe_profile_ms(res, ms, 2);
        if (st == HFE_OK) vbest[v] = std::min(vbest[v], ms[1]);
      }
      hfe_free(res);
    }
  }
  int best_v = 0;
  for (int v = 1; v < nv; ++v)
    if (vbest[v] < vbest[best_v]) best_v = v;
  g_i8_variant.store(saved_variant);
  g_profile.store(saved_profile);
  if (st != HFE_OK) return st;
  {
    std::lock_guard<std::mutex> l(g_tune_mu);
    g_tuned[{Qc->level, d3_bucket(Qc->d3)}] = best_v;
  }
  *best = best_v;
  return HFE_OK;
}

hfe_status hfe_probe_rate(int32_t which, int64_t iters, void* stream, double* rate) {
  if (!rate) return fail(HFE_EINVAL, "rate is NULL");
  *rate = 0;
  if (which < HFE_PROBE_MFMA_I8 || which > HFE_PROBE_VALU_MAD_U64) return fail(HFE_EINVAL, "unknown probe");
  if (iters < 1) return fail(HFE_EINVAL, "iters must be positive");
  hipStream_t s = (hipStream_t)stream;
  const bool valu = which == HFE_PROBE_VALU_MAD_U64;
  const int grid = device_cus() * (valu ? 8 : 4);
  DevBuf sink;
  HFE_TRY(sink.alloc((size_t)grid * 256 * 8, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hfe_status st = HFE_OK;
  float ms = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(HFE_EDEVICE, "event creation failed");
  if (st == HFE_OK) {
    hipError_t e = launch_probe(which, iters / 8 + 1, grid, sink.ptr, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_probe(which, iters, grid, sink.ptr, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) st = hip_fail(e, "rate probe");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != HFE_OK) return st;
  // MFMA: 4 waves per workgroup, 128 products of 32 x 32 x 32 per trip, 2 operations per
  // multiply-add; VALU: 64 multiply-adds per lane per trip
  const double ops = valu ? (double)grid * 256 * iters * 64 : (double)grid * 4 * iters * 128 * 32768.0 * 2;
  *rate = ms > 0 ? ops / (ms * 1e-3) : 0.0;
  return HFE_OK;
}

hfe_status hfe_autotune_save(const char* path) {
  if (!path) return fail(HFE_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(HFE_EINVAL, std::string("cannot write ") + path);
  std::lock_guard<std::mutex> l(g_tune_mu);
  for (const auto& kv : g_tuned)
    std::fprintf(f, "%d %lld %s\n", kv.first.first, (long long)kv.first.second, i8_variant_name(kv.second));
  std::fclose(f);
  return HFE_OK;
}

hfe_status hfe_autotune_load(const char* path) {
  if (!path) return fail(HFE_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(HFE_EINVAL, std::string("cannot read ") + path);
  int level;
  long long bucket;
  char name[64];
  std::map<std::pair<int, int64_t>, int> table;
  while (std::fscanf(f, "%d %lld %63s", &level, &bucket, name) == 3) {
    int v = -1;
    for (int i = 0; i < i8_variant_count(); ++i)
      if (std::string(i8_variant_name(i)) == name) v = i;
    if (v < 0) {
      std::fclose(f);
      return fail(HFE_EINVAL, std::string("unknown tile configuration ") + name);
    }
    table[{level, (int64_t)bucket}] = v;
  }
  std::fclose(f);
  std::lock_guard<std::mutex> l(g_tune_mu);
  for (const auto& kv : table) g_tuned[kv.first] = kv.second;
  return HFE_OK;
}

// ------------------------------------------------------------------ decryption
}  // extern "C"

// Decryption into caller-provided scratch y ([level][d3][rows] uint64); no allocation.
hfe_status hfe::decrypt_impl(const hfe_keys* K, const hfe_rct* R, double* v, int32_t* ip, uint64_t* y,
                               hipStream_t s) {
  const hfe_params& P = K->P;
  const int64_t ndb = 1ll << P.log_n_db;
  const int level = R->level;
  const bool ch = K->family != 0;  // n^2 chain: moduli cmod, secret products through the NTT prime
  for (int i = 0; i < level; ++i)
    HFE_LAUNCH(launch_dec_products(R->outp + (size_t)i * R->d3 * R->R_out, R->d3, R->R_out, R->row0, R->rows,
                                   (int)P.log_n_db, K->tab_db[ch ? 0 : i].tab,
                                   K->sdb_hat.as<uint64_t>() + (size_t)(ch ? 0 : i) * K->k_db * 2 * ndb, K->k_db,
                                   y + (size_t)i * R->d3 * R->rows, s, ch ? &K->cmod[i] : nullptr));
  DecodeArgs da;
  std::memset(&da, 0, sizeof(da));
  da.level = level;
  uint64_t qs[HFE_MAX_QPRIMES];
  for (int i = 0; i < level; ++i) {
    qs[i] = ch ? K->cmod[i].q : K->primes[i];
    da.q[i] = qs[i];
    da.mu[i] = ch ? K->cmod[i].mu : K->mods[i].mu;
  }
  garner_consts_of(qs, level, da.garner, da.half_digits);
  da.small = ch ? 1 : 0;
  if (ch)
    for (int i = 0; i < level; ++i) da.magic[i] = magic_u32((uint32_t)qs[i]);
  Big Q(1);
  for (int i = 0; i < level; ++i) Q.mul(qs[i]);
  for (size_t j = 0; j < 5 && j < Q.w.size(); ++j) da.Qw[j] = Q.w[j];
  da.delta_log = delta_log(K, level);
  HFE_LAUNCH(launch_decode(y, R->d3 * R->rows, da, v, ip, s));
  return HFE_OK;
}

extern "C" {

hfe_status hfe_decrypt(const hfe_keys* keys, const hfe_rct* r, double* v, int32_t* ip, void* stream) {
  const hfe_keys* K = as_handle<hfe_keys>(keys, kKeys);
  const hfe_rct* R = as_handle<hfe_rct>(r, kRct);
  if (!K || !R || !ip) return fail(HFE_EINVAL, "invalid keys, result or ip");
  if (R->keys != K) return fail(HFE_EINVAL, "result was not produced under these keys");
  hipStream_t s = (hipStream_t)stream;
  const int64_t ndb = 1ll << K->P.log_n_db;
  if ((R->row0 + R->rows - 1) / ndb >= K->k_db) return fail(HFE_ESHAPE, "rows beyond the database secrets");
  DevBuf y;
  HFE_TRY(y.alloc(sizeof(uint64_t) * (size_t)R->level * R->d3 * R->rows, s));
  return decrypt_impl(K, R, v, ip, y.as<uint64_t>(), s);
}

// ------------------------------------------------------------------ match
hfe_status hfe_match(const int32_t* ip, const uint8_t* q_masks, int64_t n_eyes, const int32_t* shifts,
                     int32_t n_shifts, const uint8_t* db_masks, int64_t rows, int32_t d2, uint32_t t_num,
                     uint32_t t_den, uint8_t* decision, uint8_t* eye_match, void* stream) {
  if (!ip || !q_masks || !shifts || !db_masks || !eye_match) return fail(HFE_EINVAL, "NULL argument");
  if (n_eyes < 1 || rows < 1 || d2 < 1) return fail(HFE_ESHAPE, "bad sizes");
  if (n_shifts < 1 || n_shifts > 64) return fail(HFE_EINVAL, "n_shifts must be 1..64");
  if (t_den == 0 || 2ull * t_num >= t_den) return fail(HFE_EINVAL, "threshold must satisfy 0 <= t < 1/2");
  hipStream_t s = (hipStream_t)stream;
  const int64_t W = (d2 + 63) / 64, d3 = n_eyes * n_shifts, nb = (rows + 255) / 256;
  DevBuf qw, dbw, part;
  HFE_TRY(qw.alloc(sizeof(uint64_t) * (size_t)W * d3, s));
  HFE_TRY(dbw.alloc(sizeof(uint64_t) * (size_t)W * rows, s));
  HFE_TRY(part.alloc((size_t)d3 * nb, s));
  HFE_LAUNCH(launch_match(ip, q_masks, n_eyes, shifts, n_shifts, db_masks, rows, d2, t_num, t_den,
                          qw.as<uint64_t>(), dbw.as<uint64_t>(), decision, part.as<uint8_t>(), eye_match, s));
  return HFE_OK;
}

// ------------------------------------------------------------------ export / shape / free
static hfe_status copy_out(const void* dev, void* dst, size_t bytes) {
  HFE_LAUNCH(hipDeviceSynchronize());
  HFE_LAUNCH(hipMemcpy(dst, dev, bytes, hipMemcpyDeviceToHost));
  return HFE_OK;
}

hfe_status hfe_export(const void* handle, int32_t which, size_t offset, uint64_t* dst, size_t n,
                      size_t* count) {
  if (!handle) return fail(HFE_EINVAL, "handle is NULL");
  const uint32_t kind = static_cast<const HandleBase*>(handle)->kind;
  size_t total = 0;
  const void* dev = nullptr;
  const int8_t* host8 = nullptr;
  if (kind == kKeys) {
    const hfe_keys* K = static_cast<const hfe_keys*>(handle);
    if (which != 0 && which != 1) return fail(HFE_EINVAL, "keys export: which must be 0 or 1");
    const std::vector<int8_t>& src = which == 0 ? K->s_host : K->sdb_host;
    total = src.size();
    host8 = src.data();
  } else if (kind == kDb) {
    const hfe_db* D = static_cast<const hfe_db*>(handle);
    if (which != 0) return fail(HFE_EINVAL, "db export: which must be 0");
    total = (size_t)D->slots_plain * D->R * D->K;
    dev = D->Dt.ptr;
    if (dst && !dev) return fail(HFE_EINVAL, "database kept no uint64 residues (plain form not requested)");
  } else if (kind == kFsKeys) {
    const hfe_fskeys* F = static_cast<const hfe_fskeys*>(handle);
    if (which != 0 && which != 1) return fail(HFE_EINVAL, "FormatSwitch keys export: which must be 0 or 1");
    const std::vector<int8_t>& src = which == 0 ? F->st_host : F->sr_host;
    total = src.size();
    host8 = src.data();
  } else if (kind == kFoldKeys) {
    const hfe_foldkeys* F = static_cast<const hfe_foldkeys*>(handle);
    if (which != 0) return fail(HFE_EINVAL, "fold keys export: which must be 0");
    total = F->s_host.size();
    host8 = F->s_host.data();
  } else if (kind == kFct) {
    const hfe_fct* X = static_cast<const hfe_fct*>(handle);
    if (which != 0) return fail(HFE_EINVAL, "fold ciphertext export: which must be 0");
    total = (size_t)X->count * 2 * (X->level + 1) * ((size_t)1 << X->keys->C.logn);
    if (count) *count = total;
    if (!dst) return HFE_OK;
    if (offset > total || n > total - offset) return fail(HFE_ESHAPE, "export range outside the array");
    DevBuf tmp;
    HFE_TRY(fold_export(X, tmp, X->stream));
    return copy_out(tmp.as<uint64_t>() + offset, dst, n * sizeof(uint64_t));
  } else if (kind == kQct) {
    const hfe_qct* Q = static_cast<const hfe_qct*>(handle);
    if (which != 0) return fail(HFE_EINVAL, "qct export: which must be 0");
    total = (size_t)Q->level * Q->d3 * Q->K;
    dev = Q->XT.ptr;
  } else if (kind == kRct) {
    const hfe_rct* R = static_cast<const hfe_rct*>(handle);
    if (which != 0) return fail(HFE_EINVAL, "rct export: which must be 0");
    total = (size_t)R->level * R->d3 * R->R_out;
    dev = R->outp;
  } else {
    return fail(HFE_EINVAL, "unknown handle");
  }
  if (count) *count = total;
  if (!dst) return HFE_OK;
  if (offset > total || n > total - offset) return fail(HFE_ESHAPE, "export range outside the array");
  if (host8) {
    for (size_t i = 0; i < n; ++i) dst[i] = (uint64_t)(int64_t)host8[offset + i];
    return HFE_OK;
  }
  return copy_out(static_cast<const uint64_t*>(dev) + offset, dst, n * sizeof(uint64_t));
}

hfe_status hfe_shape(const void* handle, int64_t* dims) {
  if (!handle || !dims) return fail(HFE_EINVAL, "NULL argument");
  const uint32_t kind = static_cast<const HandleBase*>(handle)->kind;
  if (kind == kKeys) {
    const hfe_keys* K = static_cast<const hfe_keys*>(handle);
    dims[0] = K->family ? K->cq : K->L;
    dims[1] = K->k;
    dims[2] = K->k_db;
    dims[3] = (int64_t)K->P.d2 + (1ll << K->P.log_n_q);
  } else if (kind == kDb) {
    const hfe_db* D = static_cast<const hfe_db*>(handle);
    dims[0] = D->keys->family ? D->keys->cq : D->keys->L;
    dims[1] = D->d1;
    dims[2] = D->R;
    dims[3] = D->K;
  } else if (kind == kFsKeys) {
    const hfe_fskeys* F = static_cast<const hfe_fskeys*>(handle);
    dims[0] = F->C.level;
    dims[1] = F->C.logn_t;
    dims[2] = F->C.rho;
    dims[3] = F->C.k;
  } else if (kind == kFoldKeys) {
    const hfe_foldkeys* F = static_cast<const hfe_foldkeys*>(handle);
    dims[0] = F->C.logn;
    dims[1] = F->k;
    dims[2] = F->rho;
    dims[3] = (int64_t)F->amounts.size();
  } else if (kind == kFct) {
    const hfe_fct* X = static_cast<const hfe_fct*>(handle);
    dims[0] = X->level;
    dims[1] = X->count;
    dims[2] = 1ll << X->keys->C.logn;
    dims[3] = (int64_t)X->scale;
  } else if (kind == kQct) {
    const hfe_qct* Q = static_cast<const hfe_qct*>(handle);
    dims[0] = Q->level;
    dims[1] = Q->d3;
    dims[2] = 0;
    dims[3] = Q->K;
  } else if (kind == kRct) {
    const hfe_rct* R = static_cast<const hfe_rct*>(handle);
    dims[0] = R->level;
    dims[1] = R->d3;
    dims[2] = R->rows;
    dims[3] = R->R_out;
  } else {
    return fail(HFE_EINVAL, "unknown handle");
  }
  return HFE_OK;
}

void hfe_free(void* handle) {
  if (!handle) return;
  HandleBase* b = static_cast<HandleBase*>(handle);
  switch (b->kind) {
    case kKeys:
      b->kind = 0;
      delete static_cast<hfe_keys*>(handle);
      break;
    case kDb:
      b->kind = 0;
      delete static_cast<hfe_db*>(handle);
      break;
    case kQct:
      b->kind = 0;
      delete static_cast<hfe_qct*>(handle);
      break;
    case kRct:
      if (static_cast<hfe_rct*>(handle)->is_view) break;  // owned by its plan
      b->kind = 0;
      delete static_cast<hfe_rct*>(handle);
      break;
    case kPlan:
      b->kind = 0;
      delete static_cast<hfe_plan*>(handle);
      break;
    case kServer:
      destroy_server(handle);
      break;
    case kFsKeys:
      b->kind = 0;
      delete static_cast<hfe_fskeys*>(handle);
      break;
    case kFoldKeys:
      b->kind = 0;
      delete static_cast<hfe_foldkeys*>(handle);
      break;
    case kFct:
      b->kind = 0;
      delete static_cast<hfe_fct*>(handle);
      break;
    default:
      break;
  }
}

}  // extern "C"
