// Elementwise and layout kernels around the contraction: masked ternary encoding, int8
// transpose, digit split of the database, centered CRT lift of the query with its digit
// split, rescale by the special prime, CRT decode, and the plaintext match decision.
#include "hfe_device.h"

namespace hfe {

constexpr int kMaxShifts = 64;
struct Shifts {
  int32_t r[kMaxShifts];
};

// ------------------------------------------------------------------ encode (Section 2.1.3)
// out[(e * S + s) * d2 + t] = m' - 2 (c' AND m'), c' and m' = row e rolled by shifts[s].
__global__ void k_encode(const uint8_t* codes, const uint8_t* masks, int64_t n, int32_t d2,
                         Shifts sh, int32_t n_shifts, int8_t* out) {
  const int64_t row = blockIdx.y;               // e * S + s
  const int64_t e = row / n_shifts;
  const int32_t r = sh.r[row % n_shifts];
  const uint8_t* c = codes + e * d2;
  const uint8_t* m = masks + e * d2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < d2;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t src = (t - r) % d2;
    if (src < 0) src += d2;
    const int cm = c[src] & m[src] & 1;
    out[row * d2 + t] = (int8_t)((m[src] & 1) - 2 * cm);
  }
}

// Input check of a ternary matrix: flag[0] |= 1 if any of its n entries lies outside {-1, 0, 1}.
// Thread: 16 entries (one 16-byte load when m is 16-byte aligned), grid-stride.
__global__ void __launch_bounds__(256) k_check_ternary(const int8_t* m, int64_t n, uint32_t* flag) {
  const bool vec = (reinterpret_cast<uintptr_t>(m) & 15) == 0;
  uint32_t bad = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16; i < n;
       i += (int64_t)gridDim.x * blockDim.x * 16) {
    if (vec && i + 16 <= n) {
      const uint4 w = *reinterpret_cast<const uint4*>(m + i);
      const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        // byte b is in {-1, 0, 1} iff u = b + 1 (mod 256) is in {0, 1, 2}: no bit above bit 1, and
        // not bits 0 and 1 together (u = 3); the per-byte increment carries into bit 7 at most
        const uint32_t u = ((v[k] & 0x7f7f7f7fu) + 0x01010101u) ^ (v[k] & 0x80808080u);
        bad |= (u & 0xfcfcfcfcu) | (u & (u >> 1) & 0x01010101u);
      }
    } else {
      for (int64_t j = i; j < n && j < i + 16; ++j) bad |= (uint32_t)(m[j] < -1 || m[j] > 1);
    }
  }
  if (bad) atomicOr(flag, 1u);
}

hipError_t launch_check_ternary(const int8_t* m, int64_t n, uint32_t* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 16 * 256 - 1) / (16 * 256), 4096);
  hipLaunchKernelGGL(k_check_ternary, dim3((unsigned)blocks), dim3(256), 0, s, m, n, flag);
  return hipGetLastError();
}

hipError_t launch_encode(const uint8_t* codes, const uint8_t* masks, int64_t n, int32_t d2,
                         const int32_t* shifts, int32_t n_shifts, int8_t* out, hipStream_t s) {
  if (n <= 0 || d2 <= 0) return hipSuccess;
  if (n_shifts < 1 || n_shifts > kMaxShifts) return hipErrorInvalidValue;
  Shifts sh{};
  for (int i = 0; i < n_shifts; ++i) sh.r[i] = shifts[i];
  dim3 grid((unsigned)((d2 + 255) / 256), (unsigned)(n * n_shifts));
  hipLaunchKernelGGL(k_encode, grid, dim3(256), 0, s, codes, masks, n, d2, sh, n_shifts, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ int8 transpose
__global__ void k_transpose_i8(const int8_t* in, int64_t rows, int64_t cols, int8_t* out) {
  __shared__ int8_t tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  for (int y = threadIdx.y; y < 64; y += blockDim.y) {
    const int64_t r = r0 + y, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[y][threadIdx.x] = in[r * cols + c];
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 64; y += blockDim.y) {
    const int64_t c = c0 + y, r = r0 + threadIdx.x;
    if (r < rows && c < cols) out[c * rows + r] = tile[threadIdx.x][y];
  }
}

hipError_t launch_transpose_i8(const int8_t* in, int64_t rows, int64_t cols, int8_t* out,
                               hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
  hipLaunchKernelGGL(k_transpose_i8, grid, dim3(64, 4), 0, s, in, rows, cols, out);
  return hipGetLastError();
}

// Thread (row r, block kb): 64 residues Dt[kb*64 + kk][r] -> 64 bytes of each digit plane.
__global__ void __launch_bounds__(256) k_split_db(const uint64_t* Dt, int64_t K, int64_t R, int64_t KB,
                                                  int64_t R_pad, uint64_t q, int8_t* dig) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kb = blockIdx.y;
  if (r >= R_pad) return;
  uint32_t w[kDigits][kKB / 4];
#pragma unroll
  for (int t = 0; t < kDigits; ++t)
#pragma unroll
    for (int i = 0; i < kKB / 4; ++i) w[t][i] = 0;
#pragma unroll
  for (int kk = 0; kk < kKB; ++kk) {
    const int64_t k = kb * kKB + kk;
    int64_t x = 0;
    if (r < R && k < K) x = centered(Dt[k * R + r], q);
    int32_t d[kDigits];
    split5(x, d);
#pragma unroll
    for (int t = 0; t < kDigits; ++t) w[t][kk >> 2] |= ((uint32_t)(d[t] & 255)) << (8 * (kk & 3));
  }
#pragma unroll
  for (int t = 0; t < kDigits; ++t) {
    uint4* dst = reinterpret_cast<uint4*>(dig + (((int64_t)t * KB + kb) * R_pad + r) * kKB);
#pragma unroll
    for (int i = 0; i < kKB / 16; ++i)
      dst[i] = make_uint4(w[t][4 * i], w[t][4 * i + 1], w[t][4 * i + 2], w[t][4 * i + 3]);
  }
}

hipError_t launch_split_db(const uint64_t* Dt_prime, int64_t K, int64_t R, int64_t KB, int64_t R_pad,
                           uint64_t q, int8_t* dig_prime, hipStream_t s) {
  dim3 grid((unsigned)((R_pad + 255) / 256), (unsigned)KB);
  hipLaunchKernelGGL(k_split_db, grid, dim3(256), 0, s, Dt_prime, K, R, KB, R_pad, q, dig_prime);
  return hipGetLastError();
}

// ------------------------------------------------------------------ query lift + digit split
// Element (c, k): residues XT[i][c][k] of L(x) mod q_i, where the lift L(x) is the centered CRT
// value in (-Q/2, Q/2).  Writes Xp[c][k] = L mod p (plain form) and, for every prime of the level
// and p, the 5 digit planes of the centered residue (i8 form), zero in the padding.  The K-range
// KB * 64 is a multiple of the block, so lane quads are whole.
__global__ void __launch_bounds__(256) k_lift(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB,
                                              int64_t d3_pad, LiftArgs la, uint64_t* Xp, int8_t* Xd) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= KB * kKB) return;
  lift_lane(XT, d3, K, KB, d3_pad, la, 0, Xp, Xd, blockIdx.y, k);
}

hipError_t launch_lift(const uint64_t* XT, int64_t d3, int64_t K, int64_t KB, int64_t d3_pad,
                       const LiftArgs& la, uint64_t* Xp, int8_t* Xd, hipStream_t s) {
  const int64_t kpad = KB * kKB;
  const int64_t cols = Xd ? d3_pad : d3;
  dim3 grid((unsigned)((kpad + 255) / 256), (unsigned)cols);
  hipLaunchKernelGGL(k_lift, grid, dim3(256), 0, s, XT, d3, K, KB, d3_pad, la, Xp, Xd);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rescale by p
// out[i][e] = (C[i][e] - centered(Cp[e]) mod q_i) * p^-1 mod q_i = RS_p of the CRT value.
__global__ void k_rescale(const uint64_t* C, const uint64_t* Cp, int64_t n, RescaleArgs ra,
                          uint64_t* out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    rescale_element(C, Cp, n, ra, out, e, n);
}

hipError_t launch_rescale(const uint64_t* C, const uint64_t* Cp, int64_t n, const RescaleArgs& ra,
                          uint64_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_rescale, dim3((unsigned)blocks), dim3(256), 0, s, C, Cp, n, ra, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ CRT decode
// y residues [level][n] -> Y centered in (-Q/2, Q/2) as a 320-bit two's complement integer,
// ip = floor(Y / 2^s + 1/2) and v = Y / 2^s.
__global__ void k_decode(const uint64_t* y, int64_t n, DecodeArgs da, double* v, int32_t* ip) {
  // every array below is indexed by compile-time constants (loops unrolled to the maximum level,
  // guarded by the actual one), so it stays in registers
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t r[HFE_MAX_QPRIMES] = {}, g[HFE_MAX_QPRIMES] = {};
#pragma unroll
    for (int i = 0; i < HFE_MAX_QPRIMES; ++i)
      if (i < da.level) r[i] = y[(int64_t)i * n + e];
    if (da.small)
      garner_digits_u16(r, da.level, da.garner, da.q, da.magic, g);
    else
      garner_digits(r, da.level, da.garner, da.q, da.mu, g);
    // Horner: Y = g_{l-1}; Y = Y * q_i + g_i for i = l-2 .. 0 (5 words, little endian)
    uint64_t w[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < HFE_MAX_QPRIMES; ++i)
      if (i == da.level - 1) w[0] = g[i];
#pragma unroll
    for (int i = HFE_MAX_QPRIMES - 2; i >= 0; --i) {
      if (i > da.level - 2) continue;
      uint64_t carry = g[i];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const uint64_t lo = w[j] * da.q[i];
        const uint64_t hi = mulhi64(w[j], da.q[i]);
        const uint64_t sm = lo + carry;
        carry = hi + (sm < lo ? 1 : 0);
        w[j] = sm;
      }
    }
    if (above_half(g, da.half_digits, da.level)) {  // Y -= Q
      uint64_t borrow = 0;
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const uint64_t x = w[j], q = da.Qw[j];
        const uint64_t d = x - q - borrow;
        borrow = (x < q || (x == q && borrow)) ? 1 : 0;
        w[j] = d;
      }
    }
    const bool neg = (int64_t)w[4] < 0;
    // v = Y / 2^s
    uint64_t m[5];
    if (neg) {
      uint64_t carry = 1;
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        m[j] = ~w[j] + carry;
        carry = (carry && m[j] == 0) ? 1 : 0;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 5; ++j) m[j] = w[j];
    }
    double mag = 0.0;
#pragma unroll
    for (int j = 4; j >= 0; --j) mag = mag * 18446744073709551616.0 + (double)m[j];
    if (v) v[e] = ldexp(neg ? -mag : mag, -da.delta_log);
    // ip = (Y + 2^(s-1)) >> s, arithmetic
    const int s = da.delta_log;
    const int aw = (s - 1) >> 6;
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const uint64_t add = (s > 0 && j == aw) ? 1ull << ((s - 1) & 63) : 0;
      const uint64_t x = w[j] + add;
      const uint64_t c1 = x < w[j] ? 1 : 0;
      const uint64_t b2 = x + carry;
      const uint64_t c2 = b2 < x ? 1 : 0;
      w[j] = b2;
      carry = c1 | c2;
    }
    const int wi = s >> 6, bi = s & 63;
    uint64_t lo = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      if (j == wi) lo |= w[j] >> bi;
      if (bi && j == wi + 1) lo |= w[j] << (64 - bi);
    }
    ip[e] = (int32_t)(uint32_t)lo;
  }
}

hipError_t launch_decode(const uint64_t* y, int64_t n, const DecodeArgs& da, double* v, int32_t* ip,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_decode, dim3((unsigned)blocks), dim3(256), 0, s, y, n, da, v, ip);
  return hipGetLastError();
}

// ------------------------------------------------------------------ match decision
// Masks packed into 64-bit words, words-major ([word][row]) so that a row block reads
// contiguous words.  Query masks are rolled by their shifts while packing.
// Thread (word w, row): out[w][row] = bits t = 64 w .. 64 w + 63 of the row rolled by its shift
// (bit b = mask[(t - r) mod d2] & 1, zero beyond d2).  Lanes take consecutive rows of one word,
// so the word-major writes are coalesced; an unshifted row whose 64 bytes lie inside the mask row
// is read as four 16-byte loads (one aligned 64-byte line when d2 is a multiple of 64).
__global__ void k_pack_masks(const uint8_t* masks, int64_t n, int32_t d2, Shifts sh, int32_t n_shifts,
                             int32_t W, uint64_t* out) {
  const int64_t rows = n * n_shifts;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * W) return;
  const int32_t w = (int32_t)(idx / rows);
  const int64_t row = idx - (int64_t)w * rows;  // e * S + s
  const int64_t e = row / n_shifts;
  const int32_t r = sh.r[row % n_shifts];
  const uint8_t* m = masks + e * d2;
  const int64_t t0 = (int64_t)w * 64;
  uint64_t word = 0;
  if (r == 0 && t0 + 64 <= d2 && (((uintptr_t)(m + t0)) & 15) == 0) {
    const uint4* p = reinterpret_cast<const uint4*>(m + t0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 v = p[i];
      const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int b = 0; b < 4; ++b) word |= (uint64_t)((d[k] >> (8 * b)) & 1u) << (16 * i + 4 * k + b);
    }
  } else {
    for (int b = 0; b < 64; ++b) {
      const int64_t t = t0 + b;
      if (t < d2) {
        int64_t src = (t - r) % d2;
        if (src < 0) src += d2;
        word |= (uint64_t)(m[src] & 1) << b;
      }
    }
  }
  out[(int64_t)w * rows + row] = word;
}

constexpr int kMatchCols = 16;

// Block (column group g, row block): thread = one database row, kMatchCols query columns.
__global__ void __launch_bounds__(256)
k_match(const int32_t* ip, const uint64_t* qwords, const uint64_t* dbwords, int64_t d3, int64_t rows,
        int32_t W, uint32_t t_num, uint32_t t_den, uint8_t* decision, uint8_t* part) {
  extern __shared__ uint64_t qw[];  // [kMatchCols][W]
  __shared__ int any_flag[kMatchCols];
  const int64_t c0 = (int64_t)blockIdx.y * kMatchCols;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = threadIdx.x; i < kMatchCols * W; i += blockDim.x) {
    const int cc = i / W, w = i % W;
    qw[i] = (c0 + cc < d3) ? qwords[(int64_t)w * d3 + c0 + cc] : 0ull;
  }
  if (threadIdx.x < kMatchCols) any_flag[threadIdx.x] = 0;
  __syncthreads();
  int ov[kMatchCols];
#pragma unroll
  for (int cc = 0; cc < kMatchCols; ++cc) ov[cc] = 0;
  if (r < rows) {
    for (int w = 0; w < W; ++w) {
      const uint64_t dw = dbwords[(int64_t)w * rows + r];
#pragma unroll
      for (int cc = 0; cc < kMatchCols; ++cc) ov[cc] += __popcll(qw[cc * W + w] & dw);
    }
  }
  const int64_t lhs_scale = t_den, rhs_scale = (int64_t)t_den - 2 * (int64_t)t_num;
#pragma unroll
  for (int cc = 0; cc < kMatchCols; ++cc) {
    const int64_t c = c0 + cc;
    if (r < rows && c < d3) {
      const int64_t x = ip[c * rows + r];
      const bool dec = ov[cc] > 0 && x * lhs_scale > rhs_scale * ov[cc];
      if (decision) decision[c * rows + r] = dec ? 1 : 0;
      if (dec) any_flag[cc] = 1;  // benign race: every writer stores 1
    }
  }
  __syncthreads();
  if (threadIdx.x < kMatchCols && c0 + threadIdx.x < d3)
    part[(c0 + threadIdx.x) * gridDim.x + blockIdx.x] = (uint8_t)any_flag[threadIdx.x];
}

// eye_match[e] = OR of part[c][b] over its columns c and row blocks b.
__global__ void k_eye_any(const uint8_t* part, int64_t n_eyes, int32_t n_shifts, int32_t nb,
                          uint8_t* eye_match) {
  const int64_t e = blockIdx.x;
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  const int64_t total = (int64_t)n_shifts * nb;
  int mine = 0;
  for (int64_t i = threadIdx.x; i < total; i += blockDim.x) mine |= part[e * total + i];
  if (mine) flag = 1;
  __syncthreads();
  if (threadIdx.x == 0) eye_match[e] = (uint8_t)flag;
}

hipError_t launch_match(const int32_t* ip, const uint8_t* q_masks, int64_t n_eyes,
                        const int32_t* shifts, int32_t n_shifts, const uint8_t* db_masks,
                        int64_t rows, int32_t d2, uint32_t t_num, uint32_t t_den, uint64_t* qwords,
                        uint64_t* dbwords, uint8_t* decision, uint8_t* part, uint8_t* eye_match,
                        hipStream_t s) {
  if (n_shifts < 1 || n_shifts > kMaxShifts) return hipErrorInvalidValue;
  const int32_t W = (d2 + 63) / 64;
  const int64_t d3 = n_eyes * n_shifts;
  Shifts sh{}, zero{};
  for (int i = 0; i < n_shifts; ++i) sh.r[i] = shifts[i];
  hipLaunchKernelGGL(k_pack_masks, dim3((unsigned)((d3 * W + 255) / 256)), dim3(256), 0, s,
                     q_masks, n_eyes, d2, sh, n_shifts, W, qwords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pack_masks, dim3((unsigned)((rows * W + 255) / 256)), dim3(256), 0, s,
                     db_masks, rows, d2, zero, 1, W, dbwords);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)((rows + 255) / 256);
  const size_t lds = sizeof(uint64_t) * kMatchCols * W;
  if (lds > 65536) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_match),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_match, dim3(nb, (unsigned)((d3 + kMatchCols - 1) / kMatchCols)), dim3(256), lds, s,
                     ip, qwords, dbwords, d3, rows, W, t_num, t_den, decision, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eye_any, dim3((unsigned)n_eyes), dim3(256), 0, s, part, n_eyes, n_shifts,
                     (int32_t)nb, eye_match);
  return hipGetLastError();
}

}  // namespace hfe
