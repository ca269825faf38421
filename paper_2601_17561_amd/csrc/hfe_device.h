// Device-side element operations shared by the per-call and the grouped (batched) kernels:
// balanced int8 digit split, Garner mixed-radix reconstruction, the centered CRT lift of one
// query residue vector with its digit split, and the rescale of one output entry.
#pragma once

#include "hfe_internal.h"

namespace hfe {

// MFMA operand and result vectors: 16 int8 per lane (as 4 ints), 16 int32 per lane.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Contraction row r (0 .. N_DB + rows) -> database row: the A-part rows, then the shard's rows.
__device__ __forceinline__ int64_t src_row(int64_t r, int64_t n_db, int64_t row0) {
  return r < n_db ? r : r + row0;
}

// ------------------------------------------------------------------ digit split
// Centered residue x in (-q/2, q/2) -> 5 balanced base-256 digits d_t in [-128, 127]
// (|d_4| <= 8), x = sum_t d_t 256^t.
__device__ __forceinline__ void split5(int64_t x, int32_t d[kDigits]) {
#pragma unroll
  for (int t = 0; t < kDigits - 1; ++t) {
    const int32_t lo = (int32_t)((x + 128) & 255) - 128;
    d[t] = lo;
    x = (x - lo) >> 8;
  }
  d[kDigits - 1] = (int32_t)x;
}

// ------------------------------------------------------------------ direct global-to-LDS load
// global_load_lds_dwordx4: each lane's 16 bytes at g land in LDS at M0 + 16 * lane.  The load is
// counted by vmcnt like any vector load; callers wait for it with explicit s_waitcnt.  M0 is
// written and not restored: the compiler reserves M0 and sets it right before the few
// instructions that read it, so no value of its own lives in M0 across this statement (the clobber
// entry records the write; the compiler warns that it does not act on it).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const int8_t* g, uint32_t lds_addr) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(g)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// ------------------------------------------------------------------ Garner mixed radix
// Residues y_i mod q_i -> digits v_i with Y = v_0 + v_1 q_0 + v_2 q_0 q_1 + ..., computed as
// v_i = (y_i - sum_{j<i} v_j (q_0..q_{j-1} mod q_i)) * (q_0..q_{i-1})^-1 mod q_i.
// garner[i][j] = q_0..q_{j-1} mod q_i for j < i, garner[i][i] = (q_0..q_{i-1})^-1 mod q_i.
__device__ __forceinline__ void garner_digits(const uint64_t* y, int level,
                                              const uint64_t (*garner)[HFE_MAX_QPRIMES],
                                              const uint64_t* q, const uint64_t* mus, uint64_t* v) {
  // loops unrolled to the maximum level, so that y and v stay in registers
#pragma unroll
  for (int i = 0; i < HFE_MAX_QPRIMES; ++i) {
    if (i >= level) break;
    const uint64_t qi = q[i];
    const uint64_t mu = mus[i];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < i; ++j)
      s = add_mod(s, mul_mod(barrett64(v[j], qi, mu), garner[i][j], qi, mu), qi);
    v[i] = i == 0 ? y[0] : mul_mod(sub_mod(y[i], s, qi), garner[i][i], qi, mu);
  }
}

// The same digits when every modulus is at most 2^16 (the n^2 chain), in 32-bit products:
// magic[i] = ceil(2^32 / q_i), and the Garner constants below q_i.
template <class T>
__device__ __forceinline__ void garner_digits_u16(const T* y, int level, const uint64_t (*garner)[HFE_MAX_QPRIMES],
                                                  const uint64_t* q, const uint32_t* magic, T* v) {
#pragma unroll
  for (int i = 0; i < HFE_MAX_QPRIMES; ++i) {
    if (i >= level) break;
    const uint32_t qi = (uint32_t)q[i], mg = magic[i];
    uint32_t acc = 0;  // (v_0 + v_1 q_0 + ...) mod q_i
#pragma unroll
    for (int j = 0; j < i; ++j) {
      acc += mulmod_u16(mod_u32((uint32_t)v[j], qi, mg), (uint32_t)garner[i][j], qi, mg);
      acc = acc >= qi ? acc - qi : acc;
    }
    const uint32_t yi = (uint32_t)y[i];
    v[i] = i == 0 ? (T)yi : (T)mulmod_u16(yi >= acc ? yi - acc : yi + qi - acc, (uint32_t)garner[i][i], qi, mg);
  }
}

// Y > (Q - 1)/2, compared on mixed-radix digits from the most significant one.
__device__ __forceinline__ bool above_half(const uint64_t* v, const uint64_t* half, int level) {
  bool gt = false, decided = false;
#pragma unroll
  for (int i = HFE_MAX_QPRIMES - 1; i >= 0; --i) {
    if (i < level && !decided && v[i] != half[i]) {
      gt = v[i] > half[i];
      decided = true;
    }
  }
  return gt;
}

// Query element (c, k) of XT ([level][d3][K]): the residues y_i of the lift L(x) = centered
// CRT value in (-Q/2, Q/2), and lp = L mod p.  Returns false for padding positions (c >= d3 or
// k >= K), where the lifted value is 0.
__device__ __forceinline__ bool lift_residues(const uint64_t* XT, int64_t d3, int64_t K, const LiftArgs& la,
                                              int64_t c, int64_t k, uint64_t* y, uint64_t& lp) {
  lp = 0;
  if (c >= d3 || k >= K) return false;
#pragma unroll
  for (int i = 0; i < HFE_MAX_QPRIMES; ++i)
    if (i < la.level) y[i] = XT[((int64_t)i * d3 + c) * K + k];
  uint64_t v[HFE_MAX_QPRIMES] = {};
  garner_digits(y, la.level, la.garner, la.q, la.mu, v);
  const uint64_t p = la.p;
  const uint64_t mup = la.mu_p;
#pragma unroll
  for (int i = 0; i < HFE_MAX_QPRIMES; ++i)
    if (i < la.level) lp = add_mod(lp, mul_mod(barrett64(v[i], p, mup), la.mprod_p[i], p, mup), p);
  if (above_half(v, la.half_digits, la.level)) lp = sub_mod(lp, la.Q_mod_p, p);
  return true;
}

// ------------------------------------------------------------------ small-modulus constants
// The RNS moduli and n^2 bases with their reciprocals, computed at compile time (hfe_exact.h).
__constant__ static RnsModConsts kRnsC = make_rns_mod_consts();
__constant__ static P2BaseConsts kP2C = make_p2_base_consts();

// x (|x| < 2^40) -> x mod m_j in [-floor(m_j/2), ceil(m_j/2) - 1] for the modulus kRnsMods[j].
__device__ __forceinline__ int32_t balanced_mod(int64_t x, int j) {
  return balanced_mod_by(x, kRnsC.m[j], kRnsC.magic[j], kRnsC.t24[j]);
}

// Centered x (|x| < 2^48) -> the n^2-form digits (M, M') of base n = kP2Bases[j].
__device__ __forceinline__ void p2_digits(int64_t x, int j, int32_t& M, int32_t& Mp) {
  p2_digits_by(x, kP2C.n[j], kP2C.m[j], kP2C.magic_n[j], kP2C.rcp_m[j], M, Mp);
}

// The bytes b of the 4 lanes of a lane quad (lanes 4i .. 4i + 3, lane 4i + e holding byte e),
// packed into one 32-bit word that every lane of the quad receives (two DPP quad permutations).
// Every lane of the quad must be active.
__device__ __forceinline__ uint32_t quad_word(uint32_t b) {
  uint32_t v = (b & 255u) << (8 * (threadIdx.x & 3));
  v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm(1, 0, 3, 2)
  v |= (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm(2, 3, 0, 1)
  return v;
}

// Query element (c, k), computed by lane k mod 4 of a lane quad whose 4 lanes hold k - k mod 4 ..
// + 3 of the same column (whole quads active): the lift (as lift_residues; zero in the padding),
// L mod p into Xp[c][k] when Xp is given, and, when X is given, for every prime of the level and p
// the int8 planes of the centered residue, stored by the quad's first lane as one 4-byte word per
// plane: form 0 the 5 balanced digits (X[z][t][kb][c][kk]), form n > 0 the balanced residues
// modulo the first n small moduli (X[z][j][kb][c][kk]), form -n < 0 the n^2-form digits M, M' of
// the first n bases (X[z][2j + t][kb][c][kk]).
__device__ __forceinline__ void lift_lane(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                                          const LiftArgs& la, int form, uint64_t* Xp, int8_t* X, int64_t c,
                                          int64_t k) {
  uint64_t y[HFE_MAX_QPRIMES] = {};
  uint64_t lp;
  const bool valid = lift_residues(XT, d3, K, la, c, k, y, lp);
  if (valid && Xp) Xp[c * K + k] = lp;
  if (!X) return;
  const bool writer = (threadIdx.x & 3) == 0;
  const int64_t kb = k / kKB, kk = k % kKB - (k & 3);
  const int planes = form == 0 ? kDigits : form > 0 ? form : -2 * form;
  const int64_t pstride = KB * d3_pad * kKB / 4;  // words between consecutive planes
  // the planes of prime slot z (the level's primes, then p) for centered value x
  auto emit = [&](int z, int64_t x) {
    uint32_t* row = reinterpret_cast<uint32_t*>(X + (((int64_t)z * planes * KB + kb) * d3_pad + c) * kKB + kk);
    if (form == 0) {
      int32_t d[kDigits];
      split5(x, d);
#pragma unroll
      for (int t = 0; t < kDigits; ++t) {
        const uint32_t w = quad_word((uint32_t)d[t]);
        if (writer) row[t * pstride] = w;
      }
    } else if (form > 0) {
      for (int j = 0; j < form; ++j) {
        const uint32_t w = quad_word((uint32_t)balanced_mod(x, j));
        if (writer) row[j * pstride] = w;
      }
    } else {
      for (int j = 0; j < -form; ++j) {
        int32_t M, Mp;
        p2_digits(x, j, M, Mp);
        const uint32_t w0 = quad_word((uint32_t)M), w1 = quad_word((uint32_t)Mp);
        if (writer) {
          row[2 * j * pstride] = w0;
          row[(2 * j + 1) * pstride] = w1;
        }
      }
    }
  };
#pragma unroll
  for (int z = 0; z < HFE_MAX_QPRIMES; ++z) {
    if (z >= la.level) break;
    emit(z, valid ? centered(y[z], la.q[z]) : 0);
  }
  emit(la.level, valid ? centered(lp, la.p) : 0);
}


// CRT of one entry (see k_crt_rns): residues r[j n] mod m_j -> the exact centered sum mod the prime
// of database slot `slot`.
__device__ __forceinline__ uint64_t crt_entry(const uint8_t* r, int64_t n, const RnsCrtArgs& ra, int slot) {
  float frac = 0.f;
  uint64_t acc = 0;  // sum of y_j ((M/m_j) mod q) < 16 * 2^8 * 2^36
  for (int j = 0; j < ra.n; ++j) {
    const uint32_t y = mod_small((uint32_t)r[(size_t)j * n] * (uint32_t)ra.inv[j], (uint32_t)ra.m[j], ra.magic[j]);
    frac = crt_frac_add(frac, y, ra.rcp[j]);
    acc += (uint64_t)y * ra.Mj_mod_q[slot][j];
  }
  return crt_finish(acc, crt_round(frac), ra.M_mod_q[slot], ra.mod[slot]);
}

// Entries e0 .. e0 + 3 (those below n) of one prime slot: r = that slot's first residue plane
// ([n_mod][n] bytes), out = its n results.  With n a multiple of 4 the residues of each modulus
// are read as one 4-byte word and the results written as two 16-byte vectors.
// The same for n a multiple of 4, into registers: v[b] = entry e0 + b.
__device__ __forceinline__ void crt_quad_vals(const uint8_t* r, int64_t n, const RnsCrtArgs& ra, int slot,
                                              int64_t e0, uint64_t v[4]) {
  float frac[4] = {0.f, 0.f, 0.f, 0.f};
  uint64_t acc[4] = {0, 0, 0, 0};
  for (int j = 0; j < ra.n; ++j) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(r + (size_t)j * n + e0);
    const uint32_t m = (uint32_t)ra.m[j], magic = ra.magic[j], inv = (uint32_t)ra.inv[j];
    const uint64_t mj = ra.Mj_mod_q[slot][j];
    const float rcp = ra.rcp[j];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t y = mod_small(((w >> (8 * b)) & 255u) * inv, m, magic);
      frac[b] = crt_frac_add(frac[b], y, rcp);
      acc[b] += (uint64_t)y * mj;
    }
  }
  const Mod md = ra.mod[slot];
#pragma unroll
  for (int b = 0; b < 4; ++b) v[b] = crt_finish(acc[b], crt_round(frac[b]), ra.M_mod_q[slot], md);
}

__device__ __forceinline__ void crt_quad(const uint8_t* r, int64_t n, const RnsCrtArgs& ra, int slot, uint64_t* out,
                                         int64_t e0) {
  if ((n & 3) != 0) {
    for (int b = 0; b < 4 && e0 + b < n; ++b) out[e0 + b] = crt_entry(r + e0 + b, n, ra, slot);
    return;
  }
  uint64_t v[4];
  crt_quad_vals(r, n, ra, slot, e0, v);
  reinterpret_cast<ulonglong2*>(out + e0)[0] = make_ulonglong2(v[0], v[1]);
  reinterpret_cast<ulonglong2*>(out + e0)[1] = make_ulonglong2(v[2], v[3]);
}

// RS_p of one entry from its residues: c_i mod q_i for the level's primes and cp mod p.
__device__ __forceinline__ uint64_t rescale_value(uint64_t c_i, int64_t cp_centered, const RescaleArgs& ra, int i) {
  const Mod& m = ra.mod[i];
  const uint64_t d = sub_mod(c_i, from_signed(cp_centered, m.q, m.mu), m.q);
  return mul_shoup(d, ra.pinv[i], ra.pinv_sh[i], m.q);
}

// Output entry e of a contraction (C[i] = residues mod q_i, Cp = residues mod p, n entries per
// prime): out[i][e] = (C[i][e] - centered(Cp[e]) mod q_i) * p^-1 mod q_i = RS_p of the CRT value.
// zstride: distance between the C entries of consecutive primes (n when C is [level + 1][n]).
__device__ __forceinline__ void rescale_element(const uint64_t* C, const uint64_t* Cp, int64_t n,
                                                const RescaleArgs& ra, uint64_t* out, int64_t e,
                                                int64_t zstride) {
  const int64_t cp = centered(Cp[e], ra.p);
  for (int i = 0; i < ra.level; ++i) {
    const Mod& m = ra.mod[i];
    const uint64_t r = from_signed(cp, m.q, m.mu);
    const uint64_t d = sub_mod(C[(int64_t)i * zstride + e], r, m.q);
    out[(int64_t)i * n + e] = mul_shoup(d, ra.pinv[i], ra.pinv_sh[i], m.q);
  }
}

// The same for an entry whose residues sit at src + z zstride (z = 0 .. level, p last).
__device__ __forceinline__ void rescale_from(const uint64_t* src, int64_t zstride, const RescaleArgs& ra,
                                             uint64_t* out, int64_t n, int64_t e) {
  rescale_element(src - e, src - e + (int64_t)ra.level * zstride, n, ra, out, e, zstride);
}

}  // namespace hfe
