// Internal declarations of the encrypted-CCMM library: handle structs, device buffers,
// error reporting and the kernel launchers implemented in the .hip files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hfe.h"
#include "hfe_exact.h"
#include "hfe_math.h"

namespace hfe {

constexpr int kMaxPrimes = HFE_MAX_QPRIMES + 1;  // q_0..q_{L-1} and p
constexpr int kDigits = 5;                       // balanced base-256 digits per 36-bit residue
constexpr int kKB = 64;                          // K bytes per digit block
constexpr int kRowPad = 256;                     // extra zero rows after the digit planes
constexpr int kMaxLogN = 14;                     // ring degrees handled by the LDS-resident NTT
constexpr int kMaxLogNBig = 16;                  // ring degrees handled at all (two-pass NTT above 2^14)
constexpr int kXcds = 8;                         // accelerator complex dies (one L2 each) of an MI355X

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
const char* get_error();

struct Status {
  hfe_status code;
};

#define HFE_CHECK_HIP(expr)                                                        \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::hfe::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));         \
      return HFE_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define HFE_TRY(expr)                  \
  do {                                 \
    hfe_status _s = (expr);            \
    if (_s != HFE_OK) return _s;       \
  } while (0)

hfe_status fail(hfe_status code, const std::string& msg);

// ------------------------------------------------------------------ device memory
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// Owning device buffer (released in stream order on the stream it was allocated on).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    reset();
    ptr = o.ptr;
    bytes = o.bytes;
    stream = o.stream;
    o.ptr = nullptr;
    o.bytes = 0;
    return *this;
  }
  ~DevBuf() { reset(); }
  hfe_status alloc(size_t n, hipStream_t s);
  void reset();
  template <class T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

// ------------------------------------------------------------------ NTT tables
// Forward: Cooley-Tukey with psi^brv(i) twiddles (bit-reversed output); inverse:
// Gentleman-Sande with psi^-brv(i) twiddles and the 1/n scale (natural-order output).
struct NttTab {
  const double* psi_d;   // psi^brv(i) mod q, n entries (exact integers as doubles)
  const double* ipsi_d;  // psi^-brv(i) mod q
  uint64_t q;
  double qd, qinv, n_inv_d;  // q, RN(1/q), n^-1 mod q
  int logn;
};

struct NttTabOwner {
  DevBuf buf;  // psi | ipsi as doubles, n entries each
  NttTab tab{};
};

// ------------------------------------------------------------------ handles
enum Kind : uint32_t {
  kKeys = 0x4b455953, kDb = 0x44422020, kQct = 0x51435420, kRct = 0x52435420, kPlan = 0x504c414e, kServer = 0x53525652,
  kFsKeys = 0x46534b59, kFoldKeys = 0x464c4b59, kFct = 0x46435420
};

struct HandleBase {
  uint32_t kind;
  hipStream_t stream;  // stream of the work that produced the handle
};

}  // namespace hfe

struct hfe_keys : hfe::HandleBase {
  hfe_params P;
  int L;                                   // query primes carried (n_q_primes)
  int n_primes;                            // L + 1
  uint64_t primes[hfe::kMaxPrimes];        // q_0..q_{L-1}, p (index L)
  uint32_t prime_id[hfe::kMaxPrimes];      // random-stream ids (i, or 16 for p)
  hfe::Mod mods[hfe::kMaxPrimes];
  int k, k_db;
  std::vector<int8_t> s_host;              // k x N_Q
  std::vector<int8_t> sdb_host;            // k_db x N_DB
  hfe::NttTabOwner tab_db[hfe::kMaxPrimes];   // ring N_DB
  hfe::NttTabOwner tab_q[hfe::kMaxPrimes];    // ring N_Q
  hfe::DevBuf s_hat;                       // [prime][k][N_Q]: NTT(s_j), then Shoup companions
  hfe::DevBuf sconj_hat;                   // [k][N_Q] mod q_0: NTT of s~_j(X) = s_j(1/X), + Shoup
  hfe::DevBuf sdb_hat;                     // [prime][k_db][N_DB]: NTT(s'_j), + Shoup
  hfe::DevBuf cdt;                         // 19 uint64
  uint64_t cdt_host[19];
  // The n^2 modulus chain (Section 6.3): family 1.  The secrets, the tables of primes[0] (the NTT
  // prime of the exact secret products) and everything above are as for the prime family.
  int family = 0;                          // 0: 36-bit NTT primes; 1: the n^2 modulus chain
  int cq = 0, cp = 0;                      // chain: query moduli, special moduli
  int32_t cbase[24] = {};                  // chain bases n: the query bases, then the special part's
  hfe::Mod cmod[24] = {};                  // chain moduli n^2, same order
  uint64_t cP = 0;                         // chain: P, the product of the special moduli
};


struct hfe_db : hfe::HandleBase {
  const hfe_keys* keys;
  int64_t d1, R, K;                        // R = N_DB + d1 rows, K = d2 + N_Q columns
  int64_t KB;                              // ceil(K / 64) digit blocks
  int64_t R_pad;                           // rows of a digit plane (R + padding)
  uint32_t forms;
  hfe::DevBuf Dt;                          // [prime][K][R] uint64 (column-major D), plain form
  hfe::DevBuf digits;                      // [prime][5][KB][R_pad][64] int8, i8 form
  int n_rns = 0;                           // small moduli in use (RNS form)
  hfe::DevBuf rns;                         // [prime][n_rns][KB][R_pad][64] int8, RNS form
  int n_p2 = 0;                            // bases n in use (n^2 form)
  hfe::DevBuf p2;                          // [prime][2 n_p2][KB][R_pad][64] int8: M, M' per base
  // Prime slots of the plain residues and of the int8 planes: the keys' primes for the prime family;
  // for the n^2 chain, the moduli (query, then special) of Dt and one slot of n_p2 = cp + cq bases
  // (the special moduli first) for the planes.
  int slots_plain = 0, slots_planes = 0;
};

struct hfe_qct : hfe::HandleBase {
  const hfe_keys* keys;
  int level;
  int64_t d3, K;
  hfe::DevBuf XT;                          // [level][d3][K] uint64: row c = [b_c | a_c]
  hipEvent_t ev[5] = {};                   // FormatSwitch stage boundaries when profiling
  ~hfe_qct() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

struct hfe_rct : hfe::HandleBase {
  const hfe_keys* keys;
  int level;
  int64_t d3, row0, rows, R_out;           // R_out = N_DB + rows
  hfe::DevBuf out;                         // owned storage (empty for a view into a plan)
  uint64_t* outp = nullptr;                // [level][d3][R_out] uint64 residues
  bool is_view = false;                    // owned by an hfe_plan; hfe_free ignores it
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // stage boundaries when profiling
  ~hfe_rct() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace hfe {

// ------------------------------------------------------------------ host math (hfe_host.cpp)
bool is_prime_u64(uint64_t n);
uint64_t pow_mod(uint64_t a, uint64_t e, uint64_t q);
uint64_t inv_mod(uint64_t a, uint64_t q);
Mod make_mod(uint64_t q);
uint64_t shoup(uint64_t w, uint64_t q);
// psi = primitive 2n-th root of unity (g^((q-1)/2n), g the smallest generator)
uint64_t primitive_2n_root(uint64_t q, int logn);
// host tables (psi_rev, psi_rev_sh, ipsi_rev, ipsi_rev_sh) for one prime and ring degree
void ntt_tables_host(uint64_t q, int logn, std::vector<uint64_t>& out);
int cdt_table_quad_impl(uint64_t* dst);  // hfe_cdt.cpp (quad precision), 0 on success

// ------------------------------------------------------------------ launchers (.hip files)
// All launchers enqueue on `s` and return hipGetLastError() of the launch.
// Negacyclic forward NTT in place of `count` polynomials of length n = 2^tab.logn starting at
// a + i * stride; with_shoup also writes the Shoup companions at a + i * stride + n.
hipError_t launch_ntt_fwd(uint64_t* a, int64_t count, int64_t stride, NttTab tab, bool with_shoup,
                          hipStream_t s);

// T = M_DB S_Q mod q_0, centered to int32 (row-major in Trow, d1 x N_Q scratch) and
// transposed into Tt[v][i] (N_Q x d1).
hipError_t launch_db_T(const int8_t* m_db, int64_t d1, int32_t d2, const uint64_t* sconj_hat,
                       int k, NttTab tab_q0, int32_t* Trow, int32_t* Tt, hipStream_t s);

// Transposes: in (rows x cols) int8 -> out (cols x rows).
hipError_t launch_transpose_i8(const int8_t* in, int64_t rows, int64_t cols, int8_t* out,
                               hipStream_t s);

struct DbEncArgs {
  uint64_t seed;
  const int8_t* MT;         // d2 x d1 (transposed M_DB)
  const int32_t* Tt;        // N_Q x d1
  const uint64_t* cdt;
  int64_t d1, d2, K, R;
  int k_db;
  uint64_t p;
};
// Per prime: columns of D (Dt rows): [a_c (N_DB) | B[:, c] (d1)].
hipError_t launch_db_encrypt(const DbEncArgs& a, uint64_t* Dt_prime, uint32_t prime_id,
                             const Mod& m, NttTab tab_db, const uint64_t* sdb_hat_prime,
                             hipStream_t s);

struct QEncArgs {
  uint64_t seed;
  const int8_t* m_q;        // d3 x d2
  const uint64_t* cdt;
  int64_t d3, d2, K;
  int k;
  const int8_t* e = nullptr;  // the query errors e(t, c), d3 x d2, when drawn once for every prime
};
// The query errors of an encryption (stream QE, element (t, c); the same for every prime) into
// e[c][t], d3 x d2 (|e| <= 19 fits int8), two positions from each Philox block.
hipError_t launch_q_errors(uint64_t seed, const uint64_t* cdt, int64_t d3, int64_t d2, int8_t* e, hipStream_t s);
hipError_t launch_q_encrypt(const QEncArgs& a, uint64_t* XT_prime, uint32_t prime_id,
                            const Mod& m, uint64_t delta_mod, NttTab tab_q,
                            const uint64_t* s_hat_prime, hipStream_t s);

// The same operations for ring degrees above 2^14 (k_ntt_big.hip): two-pass transforms through
// device workspaces taken from the allocator; the LDS-resident launchers forward to these.
hipError_t launch_ntt_fwd_big(uint64_t* a, int64_t count, int64_t stride, NttTab tab, bool with_shoup,
                              hipStream_t s);
hipError_t launch_db_T_big(const int8_t* m_db, int64_t d1, int32_t d2, const uint64_t* sconj_hat, int k,
                           NttTab tab_q0, int32_t* Trow, hipStream_t s);
hipError_t launch_db_encrypt_big(const DbEncArgs& a, uint64_t* Dt_prime, uint32_t prime_id, const Mod& m,
                                 NttTab tab_db, const uint64_t* sdb_hat_prime, hipStream_t s);
hipError_t launch_q_encrypt_big(const QEncArgs& a, uint64_t* XT_prime, uint32_t prime_id, const Mod& m,
                                uint64_t delta_mod, NttTab tab_q, const uint64_t* s_hat_prime, hipStream_t s);
hipError_t launch_dec_products_big(const uint64_t* out_prime, int64_t d3, int64_t R_out, int64_t row0,
                                   int64_t rows, NttTab tab, const uint64_t* sdb_hat_prime, int j0, int j1,
                                   const Mod& arith, uint64_t* y_prime, hipStream_t s);

// Digit split of the database: Dt [K][R] residues mod q -> digits [5][KB][R_pad][64].
hipError_t launch_split_db(const uint64_t* Dt_prime, int64_t K, int64_t R, int64_t KB,
                           int64_t R_pad, uint64_t q, int8_t* dig_prime, hipStream_t s);

// Centered CRT lift of the query from Q_level to p, plus the int8 digit planes of every
// prime of the level and p.  XT: [level][d3][K].  Outputs: Xp [d3][K] (lift mod p, may be
// null) and Xd [level+1][5][KB][d3_pad][64] (may be null).
struct LiftArgs {
  int level;
  uint64_t q[HFE_MAX_QPRIMES];
  uint64_t mu[HFE_MAX_QPRIMES];                       // floor(2^64 / q_i)
  uint64_t p, mu_p;
  uint64_t garner[HFE_MAX_QPRIMES][HFE_MAX_QPRIMES];  // [i][j<i]: q_0..q_{j-1} mod q_i; [i][i]: inverse
  uint64_t mprod_p[HFE_MAX_QPRIMES + 1];              // q_0..q_{i-1} mod p
  uint64_t half_digits[HFE_MAX_QPRIMES];              // mixed-radix digits of (Q-1)/2
  uint64_t Q_mod_p;
};
hipError_t launch_lift(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                       const LiftArgs& la, uint64_t* Xp, int8_t* Xd, hipStream_t s);

// Small-modulus (RNS) form: the database and the lifted query as one balanced int8 plane per
// modulus (layouts as the digit planes); one int8 product per (prime, modulus) reduced mod the
// modulus into res[z][j][c][r] (one byte); the CRT of the n residues gives the exact centered
// integer sum, reduced mod the prime into C[z][c][r].
hipError_t launch_split_db_rns(const uint64_t* Dt_prime, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                               uint64_t q, int n_mod, int8_t* dig_prime, hipStream_t s);
hipError_t launch_lift_rns(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                           const LiftArgs& la, int n_mod, int8_t* Xr, hipStream_t s);
struct RnsGemmArgs {
  int nz, n_mod;
  const int8_t* Dr[kMaxPrimes];                // [n_mod][KB][R_pad][64] per prime slot
  const int8_t* Xr[kMaxPrimes];                // [n_mod][KB][d3_pad][64]
  int32_t m[kRnsMaxMods];
  uint32_t magic[kRnsMaxMods];                 // ceil(2^32 / m): x mod m by multiply-high, x < 2^24
  uint8_t* res;                                // [nz][n_mod][d3][R_out], residues < m_j <= 256
  int64_t KB, R_pad, n_db, row0, R_out, d3, d3_pad;
};
// tq: query columns of the workgroup tile, 128 or 256 (g.d3_pad a multiple of it)
hipError_t launch_gemm_rns(const RnsGemmArgs& g, int tq, hipStream_t s);
// the tile width with less padded work for problems of d3 columns, R_out rows and nz prime slots
int rns_tile_q(const int64_t* d3, const int64_t* R_out, const int* nz, int n);
struct RnsCrtArgs {
  int n;                                       // moduli in use
  int32_t m[kRnsMaxMods];
  uint32_t magic[kRnsMaxMods];                 // ceil(2^32 / m)
  int32_t inv[kRnsMaxMods];                    // (M / m_j)^-1 mod m_j, M = prod m
  float rcp[kRnsMaxMods];                      // 1 / m_j
  Mod mod[kMaxPrimes];                         // prime of each slot
  uint64_t Mj_mod_q[kMaxPrimes][kRnsMaxMods];  // (M / m_j) mod that prime
  uint64_t M_mod_q[kMaxPrimes];                // M mod that prime
};
hipError_t launch_crt_rns(const uint8_t* res, int nz, int64_t n, const RnsCrtArgs& ra, uint64_t* C,
                          hipStream_t s);
constexpr int kRnsTileR = 256, kRnsTileQ = 256;  // RNS workgroup tile: rows, widest query columns
// n^2 form: per base n_j the database and the lifted query as two balanced int8 planes, M and M'
// with x = M + n_j M' (mod n_j^2) (planes 2j and 2j + 1, layouts as the digit planes); per (prime,
// base) the products G0 = sum M N and G1 = sum (M N' + M' N) give S mod n_j^2 = G0 + n_j G1, stored
// as res[z][j][c][r] (uint16); the CRT of those residues gives the exact centered sum, reduced mod
// the prime into C[z][c][r].
hipError_t launch_split_db_p2(const uint64_t* Dt_prime, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                              uint64_t q, int n_bases, int8_t* planes_prime, hipStream_t s);
hipError_t launch_lift_p2(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                          const LiftArgs& la, int n_bases, int8_t* Xq, hipStream_t s);
constexpr int kP2TileQ = 256;  // n^2 workgroup tile: widest query columns (256 x 128 rows, or 128 x 256)
constexpr int kP2ArgBases = 16;  // bases one contraction launch takes (the n^2 chain uses up to 12)
struct P2GemmArgs {
  int nz, n_bases;
  const int8_t* Dq[kMaxPrimes];                // [2 n_bases][KB][R_pad][64] per prime slot
  const int8_t* Xq[kMaxPrimes];                // [2 n_bases][KB][d3_pad][64]
  int32_t n[kP2ArgBases], m[kP2ArgBases];      // base j: n_j and n_j^2
  double rn[kP2ArgBases], rm[kP2ArgBases];     // RN(1 / n_j), RN(1 / n_j^2)
  uint16_t* res;                               // [nz][n_bases][d3][R_out], residues < n^2
  int64_t KB, R_pad, n_db, row0, R_out, d3, d3_pad;  // d3_pad a multiple of the query tile width
};
// tq: query columns of the workgroup tile, 128 or 256 (g.d3_pad a multiple of it)
hipError_t launch_gemm_p2(const P2GemmArgs& g, int tq, hipStream_t s);
// the tile width with less padded work for problems of d3 columns, R_out rows and nz prime slots
int p2_tile_q(const int64_t* d3, const int64_t* R_out, const int* nz, int n);
struct P2CrtArgs {
  int n;                                       // bases in use
  int32_t m[kP2MaxBases];                      // n_j^2
  int32_t inv[kP2MaxBases];                    // (M / m_j)^-1 mod m_j, M = prod m
  float rcp[kP2MaxBases];                      // 1 / m_j
  Mod mod[kMaxPrimes];                         // prime of each slot
  uint64_t Mj_mod_q[kMaxPrimes][kP2MaxBases];  // (M / m_j) mod that prime
  uint64_t M_mod_q[kMaxPrimes];                // M mod that prime
};
hipError_t launch_crt_p2(const uint16_t* res, int nz, int64_t n, const P2CrtArgs& ra, uint64_t* C, hipStream_t s);

// ------------------------------------------------------------------ the n^2 modulus chain (k_chain.hip)
// Ciphertext moduli m = n^2 for primes 127 <= n <= 253 (Section 6.3): query moduli m_0..m_{L-1}, a
// special part of np moduli m'_s (the rescale divisor P = prod m'_s).  Contraction slots: the special
// moduli first (slot s), then the query moduli (slot np + j), so that a level l uses slots
// [0, np + l).
constexpr int kChainMaxP = 3;                            // P = prod m'_s < 2^48: its CRT fits 64 bits
constexpr int kChainMaxSlots = kChainMaxP + HFE_MAX_QPRIMES;
struct ChainBase {
  int32_t n, m;        // n, n^2
  uint32_t magic_n;    // ceil(2^32 / n)
  double rcp_n, rcp_m; // RN(1 / n), RN(1 / n^2)
};
ChainBase chain_base(int32_t n);
struct ChainLiftArgs {
  int level, np;
  uint64_t q[HFE_MAX_QPRIMES], mu[HFE_MAX_QPRIMES];      // query moduli m_j
  uint64_t garner[HFE_MAX_QPRIMES][HFE_MAX_QPRIMES];     // Garner constants of the query moduli
  uint64_t half_digits[HFE_MAX_QPRIMES];                 // mixed-radix digits of (Q - 1) / 2
  uint64_t pm[kChainMaxP], pmu[kChainMaxP];              // special moduli m'_s
  uint64_t mprod[kChainMaxP][HFE_MAX_QPRIMES];           // m_0 .. m_{i-1} mod m'_s
  uint64_t Q_mod[kChainMaxP];                            // Q_level mod m'_s
  uint32_t qmagic[HFE_MAX_QPRIMES], pmagic[kChainMaxP];  // ceil(2^32 / m) of the query and special moduli
  ChainBase base[kChainMaxSlots];                        // per slot
};
struct ChainRescaleArgs {
  int level, np;
  uint64_t pm[kChainMaxP], pmu[kChainMaxP];              // special moduli
  uint64_t pinv[kChainMaxP];                             // (m'_0 .. m'_{s-1})^-1 mod m'_s
  uint64_t P;                                            // prod m'_s
  Mod mod[HFE_MAX_QPRIMES];                              // query moduli
  uint64_t Pinv[HFE_MAX_QPRIMES];                        // P^-1 mod m_j
  uint32_t qmagic[HFE_MAX_QPRIMES], pmagic[kChainMaxP];  // ceil(2^32 / m)
};
// Residues Dt [K][R] mod b.m -> the slot's two planes [2][KB][R_pad][64] (M, M').
hipError_t launch_chain_split_db(const uint64_t* Dt, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                                 const ChainBase& b, int8_t* planes, hipStream_t s);
// Query residues XT [level][d3][K] -> planes Xq [slot][2][KB][d3_pad][64] of every slot.
hipError_t launch_chain_lift(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                             const ChainLiftArgs& la, int8_t* Xq, hipStream_t s);
// Contraction residues res [slot][n] (uint16, n = d3 R_out) -> RS_P, out [level][n] (uint64).
hipError_t launch_chain_rescale(const uint16_t* res, int64_t n, const ChainRescaleArgs& ra, uint64_t* out,
                                hipStream_t s);
// Contraction residues res [slot][n] -> C [level + np][n] uint64 (query moduli, then the special ones).
hipError_t launch_chain_widen(const uint16_t* res, int64_t n, int level, int np, uint64_t* C, hipStream_t s);

struct BatchDesc;
struct BatchHeader;
struct BatchElemHeader;
struct BatchCrtDesc;
// Batched RNS contraction: problem b's tiles are [tile_begin, tile_begin + rns_batched_tiles(...)),
// ordered (z, modulus, XCD-ordered tile); workgroups claim tiles per XCD as the digit form's.  The
// launch with tq = 256 serves problems [0, hdr->n_wide), the one with tq = 128 the others.
struct RnsBatchArgs {
  const BatchHeader* hdr;
  uint32_t* next;                              // hdr->next (256-column tiles)
  uint32_t* next_narrow;                       // hdr->next_narrow (128-column tiles)
  const BatchDesc* desc;
  const int8_t* Dr;                            // database planes, all slots: [slot][n_mod][KB][R_pad][64]
  int32_t n_mod, pad_;
  int32_t m[kRnsMaxMods];
  uint32_t magic[kRnsMaxMods];
  int64_t KB, R_pad;
};
int64_t rns_batched_tiles(int64_t d3, int64_t R_out, int nz, int n_mod, int tq);
hipError_t launch_gemm_rns_batched(const RnsBatchArgs& a, int grid, int tq, hipStream_t s);
// Batched n^2 contraction: problem b's tiles are [tile_begin, tile_begin + p2_batched_tiles(...)),
// ordered (z, base, XCD-ordered tile); the launch with tq = 256 serves problems [0, hdr->n_wide)
// through hdr->next, the one with tq = 128 the others through hdr->next_narrow.  Residues (uint16)
// go to desc.res.
struct P2BatchArgs {
  const BatchHeader* hdr;
  uint32_t* next;                              // hdr->next (256-column tiles)
  uint32_t* next_narrow;                       // hdr->next_narrow (128-column tiles)
  const BatchDesc* desc;
  const int8_t* Dq;                            // database planes, all slots: [slot][2 n_bases][KB][R_pad][64]
  int32_t n_bases, pad_;
  int64_t KB, R_pad;
};
int64_t p2_batched_tiles(int64_t d3, int64_t R_out, int nz, int n_bases, int tq);
hipError_t launch_gemm_p2_batched(const P2BatchArgs& a, int grid, int tq, hipStream_t s);
// ra indexed by database slot; d[b].res points at uint16 residues
hipError_t launch_crt_p2_batched(const BatchElemHeader* hdr, const BatchCrtDesc* d, const P2CrtArgs& ra, int grid,
                                 hipStream_t s);
// ra indexed by database slot (mod, Mj_mod_q, M_mod_q of slot z at [z])
hipError_t launch_crt_rns_batched(const BatchElemHeader* hdr, const BatchCrtDesc* d, const RnsCrtArgs& ra,
                                  int grid, hipStream_t s);
int rns_wgs_per_cu(int tq);

// Plain uint64 contraction.  For each prime slot z < nz: C[z][c][r] = sum_k Dt[z][k][src(r)] *
// X[z][c][k] mod prime, rows r < R_out mapped to source rows (A-part then the shard).
struct GemmArgs {
  int nz;
  const uint64_t* Dt[kMaxPrimes];
  const int8_t* Dd[kMaxPrimes];
  const uint64_t* X[kMaxPrimes];
  const int8_t* Xd[kMaxPrimes];
  uint64_t* C[kMaxPrimes];
  Mod mod[kMaxPrimes];
  int64_t K, KB, R_db, R_pad, n_db, row0, rows, R_out, d3, d3_pad;
};
hipError_t launch_gemm_plain(const GemmArgs& g, hipStream_t s);
// rate probes (k_probe.hip): which 1 = int8 MFMA on streaming random operands, 2 = on zero
// operands, 3 = v_mad_u64_u32; grid workgroups of 256 threads, sink >= grid * 256 * 8 bytes
hipError_t launch_probe(int which, int64_t iters, int grid, void* sink, hipStream_t s);
hipError_t launch_gemm_i8(const GemmArgs& g, int variant, hipStream_t s);
constexpr int kMaxI8Variants = 16;  // upper bound of i8_variant_count()
int i8_variant_count();
const char* i8_variant_name(int v);
int i8_variant_tile_rows(int v);
int i8_variant_tile_cols(int v);
int i8_variant_wgs_per_cu(int v);  // resident workgroups per CU the configuration is sized for

// Batched contraction: a device-resident table of problems sharing one database.
// A batch's problems: items with the same level and database row range are merged into one
// problem (their query columns side by side), so that only a problem, not every item, pads its
// columns to whole tiles.
struct BatchDesc {
  const int8_t* Xd;               // [nz][planes][KB][d3_pad][64] query planes of this problem
  uint64_t* C;                    // [nz][d3][R_out] contraction output
  uint8_t* res;                   // RNS form: [nz][n_mod][d3][R_out] residues by small modulus
  int64_t n_db, row0, R_out, d3;  // output row r < n_db: database row r; r >= n_db: n_db + row0 + (r - n_db)
  int64_t d3_pad;                 // columns of the query planes Xd points into (their row stride)
  int64_t tile_begin;             // first tile of this problem in the launch (multiple of 8)
  int32_t nz, pad_;
  int32_t slot[kMaxPrimes];       // database prime slot of each z
  Mod mod[kMaxPrimes];
};
struct BatchHeader {
  int64_t total_tiles;            // multiple of kXcds
  int32_t n, pad_;
  uint32_t next[kXcds];           // tiles claimed per XCD; zero in every uploaded table
  // RNS and n^2 forms: problems [0, n_wide) use 256-column query tiles (tiles [0, tiles_wide)),
  // the rest 128-column tiles, claimed by a second launch through next_narrow
  uint32_t next_narrow[kXcds];
  int64_t tiles_wide;
  int32_t n_wide, pad2_;
};
struct BatchGemmArgs {
  const BatchHeader* hdr;         // device
  uint32_t* next;                 // device, hdr->next
  const BatchDesc* desc;          // device, hdr->n entries
  const int8_t* Dd;               // database digits, all slots
  int64_t KB, R_pad;
};
int64_t i8_batched_tiles(int variant, int64_t d3, int64_t R_out, int nz);


hipError_t launch_gemm_i8_batched(const BatchGemmArgs& a, int variant, int grid, hipStream_t s);
constexpr int kQueryPad = 128;                   // query columns padded to the widest i8 tile

// Rescale by p: out[i][c][r] = (C[i][c][r] - centered(C_p[c][r])) * p^-1 mod q_i.
struct RescaleArgs {
  int level;
  Mod mod[HFE_MAX_QPRIMES];
  uint64_t pinv[HFE_MAX_QPRIMES], pinv_sh[HFE_MAX_QPRIMES];
  uint64_t p;
};
hipError_t launch_rescale(const uint64_t* C, const uint64_t* Cp, int64_t n, const RescaleArgs& ra,
                          uint64_t* out, hipStream_t s);
// Single calls of the small-modulus forms: the CRT of the residues (ra for slots 0 .. level, the
// special prime last) and the rescale by p in one pass, out[i][e] for the level's primes.
hipError_t launch_crt_rescale_rns(const uint8_t* res, int64_t n, const RnsCrtArgs& ra, const RescaleArgs& rs,
                                  uint64_t* out, hipStream_t s);
hipError_t launch_crt_rescale_p2(const uint16_t* res, int64_t n, const P2CrtArgs& ra, const RescaleArgs& rs,
                                 uint64_t* out, hipStream_t s);

// Decryption: y[i][c][r] = B_out + (s'_j * A_out)[(row0 + r) mod N_DB] mod q_i.
// arith: the modulus of the residues when it is not the table's prime (the n^2 chain; products then
// go through the table's prime, see k_ntt.hip); nullptr: the table's prime.
hipError_t launch_dec_products(const uint64_t* out_prime, int64_t d3, int64_t R_out, int64_t row0,
                               int64_t rows, int n_db_log, NttTab tab, const uint64_t* sdb_hat_prime,
                               int k_db, uint64_t* y_prime, hipStream_t s, const Mod* arith = nullptr);

struct DecodeArgs {
  int level;
  uint64_t q[HFE_MAX_QPRIMES];
  uint64_t mu[HFE_MAX_QPRIMES];
  uint64_t garner[HFE_MAX_QPRIMES][HFE_MAX_QPRIMES];
  uint64_t half_digits[HFE_MAX_QPRIMES];
  uint64_t Qw[5];           // Q as 64-bit words
  int delta_log;
  int small;                // every modulus at most 2^16 (the n^2 chain): Garner in 32-bit products
  uint32_t magic[HFE_MAX_QPRIMES];  // ceil(2^32 / q_i) when small
};
hipError_t launch_decode(const uint64_t* y, int64_t n, const DecodeArgs& da, double* v, int32_t* ip,
                         hipStream_t s);

// flag[0] |= 1 if any of the n int8 entries of m lies outside {-1, 0, 1}
hipError_t launch_check_ternary(const int8_t* m, int64_t n, uint32_t* flag, hipStream_t s);
hipError_t launch_encode(const uint8_t* codes, const uint8_t* masks, int64_t n, int32_t d2,
                         const int32_t* shifts_dev, int32_t n_shifts, int8_t* out, hipStream_t s);

hipError_t launch_match(const int32_t* ip, const uint8_t* q_masks, int64_t n_eyes,
                        const int32_t* shifts_dev, int32_t n_shifts, const uint8_t* db_masks,
                        int64_t rows, int32_t d2, uint32_t t_num, uint32_t t_den,
                        uint64_t* qwords, uint64_t* dbwords, uint8_t* decision, uint8_t* col_any,
                        uint8_t* eye_match, hipStream_t s);

constexpr int kMaxBatch = 256;                   // items per batched launch
struct BatchElemHeader {
  int64_t total;                  // elements of the launch (chunks of 256 per problem start)
  int32_t n, pad_;
};
struct BatchLiftDesc {               // one per item
  const uint64_t* XT;             // [level][d3][K] query ciphertext of the item
  int8_t* Xd;                     // its problem's [level + 1][planes][KB][d3_pad][64]
  int64_t d3, c0, cols;           // item columns, first column in the problem, columns written
                                  // (d3, plus the problem's padding for its last item)
  int64_t d3_pad, elem_begin;     // elements: cols x KB*64
  LiftArgs la;
};
struct BatchRescaleDesc {            // one per item
  // Output row r < split of column c: C + z zstride + c Ra + r (its A problem's output); rows
  // r >= split: Cb + z zstride_b + c Rb + (r - split) (its B problem's output; split = R_out and
  // Cb = C when one problem holds all its rows)
  const uint64_t* C;
  const uint64_t* Cb;
  uint64_t* out;                  // [level][n]
  int64_t n, R_out, elem_begin;   // n = d3 x R_out of the item
  int64_t split, Ra, Rb, zstride, zstride_b;
  RescaleArgs ra;
};
struct BatchCrtDesc {                // small-modulus forms, one per problem
  const uint8_t* res;             // [nz][n_mod][n] bytes (RNS form) or uint16 (n^2 form)
  uint64_t* C;                    // [nz][n]
  int64_t n, elem_begin;          // n = d3 x R_out of the problem; elements nz x n
  int32_t nz, level, pslot, pad_; // database slot of z: z < level ? z : pslot (the special prime)
};
// form: 0 = the 5-digit planes, n > 0 = the RNS form with n small moduli, -n < 0 = the n^2 form
// with n bases
hipError_t launch_lift_batched(const BatchElemHeader* hdr, const BatchLiftDesc* d, int64_t K, int64_t KB,
                               int form, int grid, hipStream_t s);
hipError_t launch_rescale_batched(const BatchElemHeader* hdr, const BatchRescaleDesc* d, int grid, hipStream_t s);

}  // namespace hfe

// A reusable batched contraction: fixed workspace and descriptor tables, so that the grouped
// launches can be captured once in a hipGraph and replayed for any batch that fits.
struct hfe_plan : hfe::HandleBase {
  const hfe_db* db = nullptr;
  int form = HFE_FORM_I8_MFMA;                         // int8 form of the plan's contraction
  int max_items = 0, max_level = 0;
  int64_t max_cols = 0;
  size_t xd_cap = 0, c_cap = 0, res_cap = 0, out_cap = 0;  // workspace capacities (bytes, elements)
  hfe::DevBuf ws_xd, ws_c, ws_res, ws_out, desc;       // device workspace and descriptor tables
  void* host_blob = nullptr;                           // pinned staging of the descriptor tables
  size_t blob_bytes = 0;
  hipEvent_t copied = nullptr;                         // staging may be rewritten after this
  // one captured graph per digit tile configuration a run has used (chosen per batch; the RNS
  // form has one configuration, index 0)
  hipGraph_t graph[hfe::kMaxI8Variants] = {};
  hipGraphExec_t exec[hfe::kMaxI8Variants] = {};
  int elem_grid = 0, n_last = 0;
  std::vector<hfe_rct*> views;
  ~hfe_plan() {
    for (int v = 0; v < hfe::kMaxI8Variants; ++v) {
      if (exec[v]) (void)hipGraphExecDestroy(exec[v]);
      if (graph[v]) (void)hipGraphDestroy(graph[v]);
    }
    if (copied) (void)hipEventDestroy(copied);
    if (host_blob) (void)hipHostFree(host_blob);
    for (auto* v : views) delete v;
  }
};

namespace hfe {
// Batch parameters of an int8 form of a database: int8 planes per prime slot, query column padding,
// bytes per residue of the small-modulus contraction (0: the contraction writes C itself), and the
// form code of the query lift (0 digits, n RNS moduli, -n n^2 bases).
struct FormShape {
  bool rns = false, p2 = false;
  int planes = 0, res_bytes = 0, lift_form = 0;
  int64_t qpad = 0;
};
FormShape form_shape(const hfe_db* D, int form);
// Decryption of a result into caller-provided scratch y ([level][d3][rows] uint64).
hfe_status decrypt_impl(const hfe_keys* K, const hfe_rct* R, double* v, int32_t* ip, uint64_t* y, hipStream_t s);
void destroy_server(void* handle);  // hfe_server.cpp
// hfe_ccmm with every device buffer of the call carved from [region, region + cap) and the
// rescaled result written to out; HFE_ENOMEM (nothing enqueued) if the call needs more.
hfe_status ccmm_region(const hfe_db* db, const hfe_qct* q, int64_t row0, int64_t rows, int32_t form,
                       hipStream_t s, uint64_t* out, void* region, size_t cap);
}  // namespace hfe

namespace hfe {
// Entries of a ternary input outside {-1, 0, 1} (they would break the bound |M m| <= d2 that the
// scale leaves room for).  begin enqueues a check kernel and the copy of its flag into a pinned
// word; the caller then enqueues its own work, and end waits for the check alone (an event after
// the copy), so the device never idles for it.  The pinned word is one per host thread, kept
// until the process ends; a call waits for it before returning, so calls never share it.
struct TernaryCheck {
  DevBuf flag;
  hipEvent_t ev = nullptr;
  uint32_t* host = nullptr;
  ~TernaryCheck() {
    if (ev) (void)hipEventDestroy(ev);
  }
};
hfe_status check_ternary_begin(const int8_t* m, int64_t n, hipStream_t s, TernaryCheck& c);
hfe_status check_ternary_end(TernaryCheck& c, const char* what);
int delta_log(const hfe_keys* k, int level);  // floor(log2(q_0 ... q_{l-1})) - gap
bool profiling();                             // hfe_profile(1) in effect
}  // namespace hfe

// ------------------------------------------------------------------ FormatSwitch (Appendix C.1)
namespace hfe {
// Stream purposes of the FormatSwitch draws: transmission secret s_T, ring-switch secret s', masks and
// errors of the ring-switching keys, of the conversion keys and of the transmission ciphertexts.
enum : uint64_t { kTSec = 7, kRSec = 8, kRkA = 9, kRkE = 10, kCkA = 11, kCkE = 12, kTxA = 13, kTxE = 14 };

// Slots of a FormatSwitch at CCMM level l: q_0 .. q_l (the transmission modulus Q'), then p.
struct FsConsts {
  int level;                     // l
  int nz;                        // l + 2
  int k;                         // chunks of N_Q code positions per query column
  int rho;                       // N_T / N_Q
  int logn_q, logn_t;
  int64_t d2;
  double zd[kMaxPrimes], zinv[kMaxPrimes];  // slot moduli and RN(1 / z)
  double ghat[kMaxPrimes];       // digit factor ((Q' / q_i) mod q_i)^-1 mod q_i, i <= l
  double pinv[kMaxPrimes];       // p^-1 mod q_i, i <= l
  double qlinv[kMaxPrimes];      // q_l^-1 mod q_i, i < l
  double scale[kMaxPrimes];      // Delta_l q_l mod q_i, i <= l (transmission scale)
  uint64_t gk[kMaxPrimes][kMaxPrimes];  // [z][i]: gadget p (Q' / q_i) mod z
  uint32_t pid[kMaxPrimes];      // random-stream id of slot z
  Mod mod[kMaxPrimes];           // slot z
  NttTab tab[kMaxPrimes];        // ring N_Q, slot z
};
}  // namespace hfe

struct hfe_fskeys : hfe::HandleBase {
  const hfe_keys* keys;
  hfe::FsConsts C;
  std::vector<int8_t> st_host;   // s_T, N_T ternary coefficients
  std::vector<int8_t> sr_host;   // s', N_Q ternary coefficients
  hfe::DevBuf st;                // s_T (int8, N_T)
  hfe::DevBuf rk;                // [z][i <= l][mask | key][rho][N_Q] doubles: NTT of the key parts, see k_fswitch.hip
  hfe::DevBuf ck;                // [z][i <= l][j < k][1 + k][N_Q] doubles: NTT of k_ij, beta_ij0 .. beta_ij(k-1)
  hfe::DevBuf st_hat;            // [i <= l][rho][N_Q] uint64: NTT of the polyphase parts of s_T
  hfe::DevBuf y_hat;             // [i <= l][N_Q] uint64: NTT of the monomial Y
  hfe::DevBuf cdt;               // the Gaussian table (19 uint64)
};

namespace hfe {
// Key material: out = [z][i][2][rho][N_Q] (rk) or [z][i][j][1 + k][N_Q] (ck) coefficient residues
// before their transforms; then the finishing passes write the doubles of the NTT-domain keys.
hipError_t launch_fs_rk_coeffs(const FsConsts& C, uint64_t seed, const int8_t* st, const uint64_t* cdt,
                               uint64_t* out, hipStream_t s);
hipError_t launch_fs_rk_finish(const FsConsts& C, const uint64_t* coef_hat, const uint64_t* sr_hat,
                               double* rk, hipStream_t s);
hipError_t launch_fs_ck_coeffs(const FsConsts& C, uint64_t seed, const int8_t* sr, const uint64_t* cdt,
                               uint64_t* out, hipStream_t s);
// s_hat: the CCMM secrets' transforms, [prime][k][2 N_Q] uint64 (values, then Shoup companions), p at
// prime index p_index.
hipError_t launch_fs_ck_finish(const FsConsts& C, const uint64_t* coef_hat, const uint64_t* s_hat, int p_index,
                               double* ck, hipStream_t s);
// Transmission encryption of ncols = d3 k ciphertexts; Ahat scratch [ncols][l + 1][rho][N_Q] doubles.
hipError_t launch_fs_tx(const FsConsts& C, uint64_t seed, const int8_t* m_q, int64_t d3, const uint64_t* st_hat,
                        const uint64_t* y_hat, const uint64_t* cdt, double* Ahat, uint64_t* T, hipStream_t s);
// The switch: digits Dg [ncols][l + 1][rho][N_Q] doubles; ring-switched Aring, Bring [nz][ncols][N_Q];
// converted Aconv [nz][d3][N_Q], Bconv [nz][d3][k][N_Q] (doubles); XT the query ciphertext.
struct FsWork {
  double* Dg;
  double* Aring;
  double* Bring;
  double* Aconv;
  double* Bconv;
};
hipError_t launch_fs_switch(const FsConsts& C, const uint64_t* T, int64_t d3, const double* rk, const double* ck,
                            const FsWork& w, uint64_t* XT, int64_t K, hipStream_t s, hipEvent_t* ev);
}  // namespace hfe

// ------------------------------------------------------------------ normalise and fold (Algorithm 2)
namespace hfe {
// Stream purposes of the fold's draws: secret positions and signs, key masks and errors, input masks
// and errors.
enum : uint64_t { kFSec = 15, kFKA = 16, kFKE = 17, kFXA = 18, kFXE = 19 };
constexpr int kFoldLevels = 4;   // q_1 .. q_4: the normalisation and three levels of f
constexpr int kFoldSlots = 6;    // q_0 .. q_4, then p
constexpr int kFoldH = 32;       // Hamming weight of the fold's secret (Appendix C.2)

struct SlotMap {
  int8_t z[kFoldSlots];          // slot position -> modulus index (0 .. 4: q_i, 5: p)
};
struct SlotFactor {
  double v[kFoldSlots];          // one residue per slot position
};
struct KeyGadget {
  double v[kFoldSlots][kFoldLevels];  // [slot position][digit]: p (Q_l / q_i) mod z
};

// An inverse transform pass of the fold (k_fold_inv): source src[item si + s ss], optionally times y at the
// same place or times pre[s]; mode 0 residues, 1 centered, 2 times f[s] (digits); dst[item di + s ds].
struct FoldInv {
  const uint64_t* src = nullptr;
  int64_t si = 0, ss = 0;
  const uint64_t* y = nullptr;
  void* dst = nullptr;
  int64_t di = 0, ds = 0;
  SlotMap zm{};
  int nsl = 0, mode = 0;
  SlotFactor f{};
  const uint64_t* pm = nullptr;          // or src times the plaintext pm[(item >> 1) pmi + z N + t] (item = 2 c + part)
  int64_t pmi = 0;
};
// A lift pass of the fold (k_fold_lift), see k_fold.hip.
struct FoldLift {
  const int64_t* cen = nullptr;          // [item][part][N] centered values of the divided-out modulus
  const uint64_t* ures = nullptr;        // or residues u mod q_cl, [item][part][N]: cen = centered(ku u mod q_cl)
  int cl = 0;
  double ku = 0.0;
  const uint64_t* x = nullptr;           // kept residues, item stride xi, part stride xp, slot stride N
  int64_t xi = 0, xp = 0;
  int has_xmul = 0;
  SlotFactor xmul{};                     // x times xmul[s] first (a constant's rescale)
  const uint64_t* add = nullptr;         // addend (ap = 0: part 0 only)
  int64_t ai = 0, ap = 0;
  const uint64_t* add2 = nullptr;        // second addend, both parts
  int64_t a2i = 0, a2p = 0;
  const uint64_t* tx = nullptr;          // tensor addend of tx, ty (item stride ti, part stride tp)
  const uint64_t* ty = nullptr;
  int64_t ti = 0, tp = 0;
  int has_tscale = 0;
  SlotFactor tscale{};                   // tensor addend times tscale[s] (a rescale by p q_l: q_l^-1)
  SlotFactor cres{};                     // constant added to part 0
  uint64_t* out = nullptr;
  int64_t oi = 0, op = 0;
  SlotMap zm{};
  int nsl = 0;
  SlotFactor inv{};
  const uint64_t* pm = nullptr;          // x times the plaintext pm[item pmi + z N + t] first (a plaintext product)
  int64_t pmi = 0;
};

struct FoldConsts {
  int logn;
  double zd[kFoldSlots], zinv[kFoldSlots];
  Mod mod[kFoldSlots];
  uint32_t pid[kFoldSlots];      // random-stream ids (i, or 16 for p)
  NttTab tab[kFoldSlots];
};
}  // namespace hfe

struct hfe_foldkeys : hfe::HandleBase {
  hfe::FoldConsts C;
  int k;                                   // folding factor
  int rho;                                 // ciphertexts per block the rotation keys cover
  std::vector<int32_t> amounts;            // rotation amounts with keys
  std::vector<int8_t> s_host;              // the secret (N ternary, weight 32)
  hfe::NttTabOwner tabs[hfe::kFoldSlots];
  hfe::DevBuf s_hat;                       // [slot][N] NTT residues of s
  hfe::DevBuf relin;                       // levels 1 .. 3, each [s][i][2][N] doubles (see k_fold.hip)
  int64_t relin_off[hfe::kFoldLevels] = {};  // offset (doubles) of the key of level l
  hfe::DevBuf rot;                         // [amount][3 slots][2 digits][2][N] doubles (level 1)
  hfe::DevBuf perm;                        // [amount][N] int32: NTT-point permutation of each rotation
  hfe::DevBuf slot_w;                      // the slot transforms' tables (hfe_slots.h): W [M/2] complex,
  hfe::DevBuf slot_z;                      // Z [M] complex (zeta^i),
  hfe::DevBuf slot_pos;                    // pos [M] int32, where slot j enters the encoder's transform,
  hfe::DevBuf slot_k;                      // k [M] int32, where the decoder's transform leaves it
  hfe::DevBuf cdt;                         // the Gaussian table
  uint64_t ksum[8] = {};                   // integer constants of f (k_0 .. k_7 as two's complement)
  double sched[8] = {};                    // S1, S2, S4, F, U, T3, T1, G
};

struct hfe_fct : hfe::HandleBase {
  const hfe_foldkeys* keys;
  int level;
  int64_t count;
  double scale;
  hfe::DevBuf ct;                          // [count][2][level + 1][N] NTT-domain residues
  hipEvent_t ev[5] = {};                   // profiled fold: start, encode, normalise, f, rotations and sums
  ~hfe_fct() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace hfe {
hipError_t launch_fold_weights(const int32_t* values, int64_t total, int mode, int64_t* w, uint32_t* bad,
                               hipStream_t s);
hipError_t launch_fold_encode(const int64_t* w, int64_t items, int logn, double scale, const double* W,
                              const double* Z, const int32_t* pos, int64_t* out, hipStream_t s);
hipError_t launch_fold_fwd(const FoldConsts& C, const int64_t* src, int64_t si, int64_t ss, uint64_t* dst, int64_t di,
                           int64_t ds, const SlotMap& zm, int nsl, int64_t items, hipStream_t s);
hipError_t launch_fold_inv(const FoldConsts& C, const FoldInv& a, int64_t items, hipStream_t s);
hipError_t launch_fold_ks_mac(const FoldConsts& C, int level, const FoldInv& dg, const uint64_t* dig, const double* keys,
                              int64_t kstride, const int32_t* kidx, uint64_t* acc, int64_t* accp, int64_t items,
                              hipStream_t s);
hipError_t launch_fold_lift(const FoldConsts& C, const FoldLift& a, int64_t items, hipStream_t s);
hipError_t launch_fold_relin_center(const FoldConsts& C, int level, const uint64_t* acc, const int64_t* accp,
                                   const uint64_t* tx, const uint64_t* ty, int64_t items, int64_t* cen, hipStream_t s);
hipError_t launch_fold_perm(const FoldConsts& C, const uint64_t* x, const int32_t* src, const int32_t* amt,
                            const int32_t* perm, uint64_t* out, int64_t items, int nsl, hipStream_t s);
hipError_t launch_fold_group_sum(const FoldConsts& C, const uint64_t* f, const uint64_t* rotated, const int32_t* beg,
                                 const int32_t* mem, uint64_t* out, int64_t groups, int nsl, hipStream_t s);
hipError_t launch_fold_scatter(const FoldConsts& C, const uint64_t* y, const int32_t* dst, uint64_t* x, int64_t items,
                               int nsl, hipStream_t s);
hipError_t launch_fold_key_coeffs(const FoldConsts& C, uint64_t seed, int kappa, int level, const SlotMap& zm,
                                  const uint64_t* cdt, uint64_t* out, hipStream_t s);
hipError_t launch_fold_key_finish(const FoldConsts& C, int level, const SlotMap& zm, const uint64_t* coef_hat,
                                  const uint64_t* s_hat, const uint64_t* from_hat, const KeyGadget& gk, double* key,
                                  hipStream_t s);
hipError_t launch_fold_add_errors(const FoldConsts& C, uint64_t seed, const uint64_t* cdt, int64_t* m, int64_t items,
                                  hipStream_t s);
hipError_t launch_fold_encrypt(const FoldConsts& C, uint64_t seed, const uint64_t* s_hat, uint64_t* ct, int64_t items,
                               hipStream_t s);
hipError_t launch_fold_dec_products(const FoldConsts& C, const uint64_t* ct, const uint64_t* s_hat, uint64_t* out,
                                    int64_t items, hipStream_t s);
hipError_t launch_fold_decode(const int64_t* m, int64_t items, int logn, const double* W, const double* Z,
                              const int32_t* kj, double inv_scale, double* v, hipStream_t s);
// Coefficient-form residues [count][2][level + 1][N] of a fold ciphertext array (hfe_export).
hfe_status fold_export(const hfe_fct* X, DevBuf& out, hipStream_t s);
}  // namespace hfe
