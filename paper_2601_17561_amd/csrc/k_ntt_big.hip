// Negacyclic NTT through HBM for ring degrees above the LDS-resident limit (2^15 and 2^16, the
// transmission ring of Appendix C.1), and the products built on it: the secret-key transforms,
// T = M_DB S_Q, database and query encryption and the decryption products of Section 2.3, with
// the same random streams, the same arithmetic and the same results as the LDS-resident kernels.
//
// The merged Cooley-Tukey transform of degree n = 2^L (twiddle psi^brv(m + i) for block i of the
// stage with m blocks, half-size t = n / 2m) splits after its first L1 = L / 2 stages:
//  * stages with t >= 2^L2 (L2 = L - L1) pair indices that agree mod 2^L2, so for each column
//    r < 2^L2 the elements r + 2^L2 k (k < 2^L1) form one transform of degree 2^L1 whose stage
//    structure and twiddle indices are those of a degree-2^L1 transform (m < 2^L1);
//  * the remaining stages pair indices inside contiguous blocks of 2^L2 elements; for block b,
//    the stage with m' local blocks has global m = 2^L1 m' and block index b m' + i', so its
//    twiddle index is m' (2^L1 + b) + i'.
// Pass 1 (columns) and pass 2 (blocks) each keep 16 sub-transforms of 256 elements in LDS and
// run the same three-stage register rounds as the LDS-resident transform, with the twiddle index
// m (mult) + i: mult = 1 in pass 1 and 2^L1 + b in pass 2.  The inverse (Gentleman-Sande) runs
// the passes in the opposite order with the same indexing and the 1/n factor at the end of
// pass 1.  NTT-domain data stays in device workspaces; only coefficient-domain results leave.
#include "hfe_internal.h"

namespace hfe {

constexpr int kBigThreads = 256;
constexpr int kBigSub = 16;                 // sub-transforms per workgroup
constexpr int64_t kBigBatchBytes = 256 << 20;  // workspace per batch of polynomials (doubles)

// ------------------------------------------------------------------ rounds over sub-arrays
// nsub sub-arrays of length nl in LDS, sub-array u at a + u * ld; mult(u) = mult0 + u * mstep.
template <int S>
__device__ __forceinline__ void fwd_round_sub(double* a, int ld, int nl, int t, int mult0, int mstep,
                                              const NttTab& T) {
  constexpr int G = 1 << S;
  const double q = T.qd, qinv = T.qinv;
  const int stride = t >> (S - 1), m1 = nl / (2 * t), gps = nl >> S;
  for (int gg = threadIdx.x; gg < kBigSub * gps; gg += blockDim.x) {
    const int u = gg / gps, g = gg - u * gps;
    double* x_base = a + u * ld;
    const int mult = mult0 + u * mstep;
    const int B = g / stride, r = g - B * stride;
    const int base = B * 2 * t + r;
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = x_base[base + k * stride];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int h = 1 << (S - 1 - s);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (k & h) continue;
        const int w = (m1 << s) * mult + (B << s) + (k >> (S - s));
        const double U = x[k];
        const double V = mulmod_d(x[k + h], T.psi_d[w], q, qinv);
        x[k] = addmod_d(U, V, q);
        x[k + h] = submod_d(U, V, q);
      }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) x_base[base + k * stride] = x[k];
  }
  __syncthreads();
}

template <int S>
__device__ __forceinline__ void inv_round_sub(double* a, int ld, int nl, int t, int mult0, int mstep,
                                              bool scale, const NttTab& T) {
  constexpr int G = 1 << S;
  const double q = T.qd, qinv = T.qinv;
  const int gps = nl >> S;
  for (int gg = threadIdx.x; gg < kBigSub * gps; gg += blockDim.x) {
    const int u = gg / gps, g = gg - u * gps;
    double* x_base = a + u * ld;
    const int mult = mult0 + u * mstep;
    const int B = g / t, r = g - B * t;
    const int base = B * G * t + r;
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = x_base[base + k * t];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int h = 1 << s;
      const int m = nl / (2 * h * t);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (k & h) continue;
        const int w = m * mult + (B << (S - 1 - s)) + (k >> (s + 1));
        const double U = x[k], V = x[k + h];
        x[k] = addmod_d(U, V, q);
        x[k + h] = mulmod_d(submod_d(U, V, q), T.ipsi_d[w], q, qinv);
      }
    }
    if (scale) {
#pragma unroll
      for (int k = 0; k < G; ++k) x[k] = mulmod_d(x[k], T.n_inv_d, q, qinv);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) x_base[base + k * t] = x[k];
  }
  __syncthreads();
}

__device__ __forceinline__ void fwd_sub(double* a, int ld, int lognl, int mult0, int mstep, const NttTab& T) {
  const int nl = 1 << lognl;
  int t = nl >> 1, left = lognl;
  while (left > 0) {
    if (left >= 3) {
      fwd_round_sub<3>(a, ld, nl, t, mult0, mstep, T);
      t >>= 3;
      left -= 3;
    } else if (left == 2) {
      fwd_round_sub<2>(a, ld, nl, t, mult0, mstep, T);
      t >>= 2;
      left -= 2;
    } else {
      fwd_round_sub<1>(a, ld, nl, t, mult0, mstep, T);
      t >>= 1;
      left -= 1;
    }
  }
}

__device__ __forceinline__ void inv_sub(double* a, int ld, int lognl, int mult0, int mstep, bool scale,
                                        const NttTab& T) {
  const int nl = 1 << lognl;
  int t = 1, left = lognl;
  while (left > 0) {
    if (left >= 3) {
      inv_round_sub<3>(a, ld, nl, t, mult0, mstep, scale && left == 3, T);
      t <<= 3;
      left -= 3;
    } else if (left == 2) {
      inv_round_sub<2>(a, ld, nl, t, mult0, mstep, scale, T);
      t <<= 2;
      left -= 2;
    } else {
      inv_round_sub<1>(a, ld, nl, t, mult0, mstep, scale, T);
      t <<= 1;
      left -= 1;
    }
  }
}

// ------------------------------------------------------------------ the two passes
// W: count polynomials of n = 2^(l1 + l2) doubles, polynomial j at W + j * n.
// Pass 1: workgroup (x, j) holds columns r = 16 x + u (u < 16), elements r + 2^l2 k (k < 2^l1),
// in LDS at u * (2^l1 + 1) + k (one padding double per column).
// Pass 2: workgroup (x, j) holds blocks b = 16 x + u, elements 2^l2 b + v (v < 2^l2), in LDS at
// u * 2^l2 + v (the global order).
template <bool kFwd>
__global__ void __launch_bounds__(kBigThreads) k_big_pass1(double* W, int l1, int l2, NttTab T) {
  extern __shared__ double lds[];
  const int nl = 1 << l1, ld = nl + 1;
  double* poly = W + ((int64_t)blockIdx.y << (l1 + l2));
  const int r0 = blockIdx.x * kBigSub;
  for (int idx = threadIdx.x; idx < kBigSub * nl; idx += blockDim.x) {
    const int k = idx / kBigSub, u = idx - k * kBigSub;
    lds[u * ld + k] = poly[r0 + u + ((int64_t)k << l2)];
  }
  __syncthreads();
  if (kFwd)
    fwd_sub(lds, ld, l1, 1, 0, T);
  else
    inv_sub(lds, ld, l1, 1, 0, true, T);
  for (int idx = threadIdx.x; idx < kBigSub * nl; idx += blockDim.x) {
    const int k = idx / kBigSub, u = idx - k * kBigSub;
    poly[r0 + u + ((int64_t)k << l2)] = lds[u * ld + k];
  }
}

template <bool kFwd>
__global__ void __launch_bounds__(kBigThreads) k_big_pass2(double* W, int l1, int l2, NttTab T) {
  extern __shared__ double lds[];
  const int nl = 1 << l2;
  double* blk = W + ((int64_t)blockIdx.y << (l1 + l2)) + ((int64_t)blockIdx.x * kBigSub << l2);
  for (int idx = threadIdx.x; idx < kBigSub * nl; idx += blockDim.x) lds[idx] = blk[idx];
  __syncthreads();
  const int mult0 = (1 << l1) + blockIdx.x * kBigSub;
  if (kFwd)
    fwd_sub(lds, nl, l2, mult0, 1, T);
  else
    inv_sub(lds, nl, l2, mult0, 1, false, T);
  for (int idx = threadIdx.x; idx < kBigSub * nl; idx += blockDim.x) blk[idx] = lds[idx];
}

static void big_split(int logn, int* l1, int* l2) {
  *l1 = logn / 2;
  *l2 = logn - *l1;
}

// Forward (kFwd) or inverse transform of `count` polynomials in W, in place.
static hipError_t big_transform(double* W, int64_t count, const NttTab& T, bool fwd, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int l1, l2;
  big_split(T.logn, &l1, &l2);
  if ((1 << l1) < kBigSub || (1 << l2) < kBigSub || l1 > 8 || l2 > 8) return hipErrorInvalidValue;
  const dim3 g1((unsigned)((1 << l2) / kBigSub), (unsigned)count), g2((unsigned)((1 << l1) / kBigSub), (unsigned)count);
  const size_t lds1 = sizeof(double) * kBigSub * ((1 << l1) + 1), lds2 = sizeof(double) * kBigSub * (1 << l2);
  if (fwd) {
    hipLaunchKernelGGL(k_big_pass1<true>, g1, dim3(kBigThreads), lds1, s, W, l1, l2, T);
    hipLaunchKernelGGL(k_big_pass2<true>, g2, dim3(kBigThreads), lds2, s, W, l1, l2, T);
  } else {
    hipLaunchKernelGGL(k_big_pass2<false>, g2, dim3(kBigThreads), lds2, s, W, l1, l2, T);
    hipLaunchKernelGGL(k_big_pass1<false>, g1, dim3(kBigThreads), lds1, s, W, l1, l2, T);
  }
  return hipGetLastError();
}

// Polynomials per batch so that one workspace of doubles stays within kBigBatchBytes.
static int64_t big_batch(int logn, int64_t total) {
  const int64_t per = std::max<int64_t>(1, kBigBatchBytes / ((int64_t)sizeof(double) << logn));
  return std::min(per, total);
}

static hipError_t ws_alloc(DevBuf& b, size_t bytes, hipStream_t s) {
  return b.alloc(bytes, s) == HFE_OK ? hipSuccess : hipErrorOutOfMemory;
}

// ------------------------------------------------------------------ element-wise kernels
// grid (ceil(n / 256), columns); element (v, column).

// Secret transforms: W[j] = a[j * stride + v] -> after the transform a[j * stride + v] = W and
// a[j * stride + n + v] = its Shoup quotient.
__global__ void k_big_load_u64(const uint64_t* a, int64_t stride, int n, double* W) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) W[(int64_t)blockIdx.y * n + v] = (double)a[(int64_t)blockIdx.y * stride + v];
}

__global__ void k_big_store_hat(const double* W, int n, uint64_t q, uint64_t* a, int64_t stride, int shoup) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t x = (uint64_t)W[(int64_t)blockIdx.y * n + v];
  a[(int64_t)blockIdx.y * stride + v] = x;
  if (shoup) a[(int64_t)blockIdx.y * stride + n + v] = shoup_quot(x, q);
}

// The n^2 modulus chain takes its products through the table's prime q (as the LDS-resident
// kernels): a residue mod m enters as its centered integer mod q, a product coefficient (an integer
// of magnitude below q / 2) leaves centered and reduced mod m.  With m = q both are identities.
__device__ __forceinline__ double big_to_ntt(uint64_t x, const Mod& M, uint64_t q) {
  if (M.q == q) return (double)x;
  const int64_t c = centered(x, M.q);
  return (double)(c >= 0 ? (uint64_t)c : q - (uint64_t)(-c));
}
__device__ __forceinline__ uint64_t big_from_ntt(double v, uint64_t q, const Mod& M) {
  if (M.q == q) return (uint64_t)v;
  return from_signed(centered((uint64_t)v, q), M.q, M.mu);
}

// Uniform a-polynomial of column c0 + y (stream key_a, element (v, c)) mod M, written to
// dst[(c0 + y) * dst_stride + v] and, as the NTT's doubles (residues mod q), to W[y].
__global__ void k_big_uniform(uint64_t seed, uint64_t key_a, Mod M, uint64_t q, int64_t c0, int n, uint64_t* dst,
                              int64_t dst_stride, double* W) {
  const int v4 = blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * v4 >= n) return;
  const int64_t c = c0 + blockIdx.y;
  const Philox4 b = philox4x64_10(seed, key_a, (uint64_t)v4, (uint64_t)c, 0, 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int v = 4 * v4 + j;
    if (v < n) {
      const uint64_t w = b.v[j];
      const uint64_t x = w < M.bound ? barrett64(w, M.q, M.mu) : uniform_at(seed, key_a, (uint64_t)v, (uint64_t)c, M);
      dst[c * dst_stride + v] = x;
      W[(int64_t)blockIdx.y * n + v] = big_to_ntt(x, M, q);
    }
  }
}

// W2[y] = W[y] . hat (pointwise mod q), or W2[y] += W[y] . hat with accumulate.
__global__ void k_big_pointwise(const double* W, const uint64_t* hat, int n, NttTab T, double* W2, int accumulate) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t o = (int64_t)blockIdx.y * n + v;
  const double x = mulmod_d(W[o], (double)hat[v], T.qd, T.qinv);
  W2[o] = accumulate ? addmod_d(W2[o], x, T.qd) : x;
}

// T rows: W[y][t] = chunk j of database row i0 + y as residues of {-1, 0, 1}.
__global__ void k_big_mdb_chunk(const int8_t* m_db, int32_t d2, int64_t i0, int j, int n, double qd, double* W) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = i0 + blockIdx.y, col = (int64_t)j * n + t;
  const int8_t m = col < d2 ? m_db[i * d2 + col] : (int8_t)0;
  W[(int64_t)blockIdx.y * n + t] = m == 1 ? 1.0 : (m == -1 ? qd - 1.0 : 0.0);
}

__global__ void k_big_store_T(const double* W, int64_t i0, int n, uint64_t q, int32_t* Trow) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  Trow[(i0 + blockIdx.y) * n + t] = (int32_t)centered((uint64_t)W[(int64_t)blockIdx.y * n + t], q);
}

// Database rows of chunk j for column c0 + y: B[i][c] = p plain[i][c] - (s'_j a_c)[i - j n] + e(i, c).
__global__ void k_big_emit_db(const double* W2, DbEncArgs A, int64_t c0, int j, int n, uint64_t* Dt, Mod M,
                              uint64_t qt, uint64_t key_e) {
  const int64_t c = c0 + blockIdx.y;
  const int64_t i = (int64_t)j * n + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.d1 || i >= (int64_t)(j + 1) * n) return;
  const uint64_t q = M.q;
  const uint64_t pm = barrett64(A.p, q, M.mu);
  const int32_t pl = c < A.d2 ? (int32_t)A.MT[c * A.d1 + i] : A.Tt[(c - A.d2) * A.d1 + i];
  const int32_t e = gaussian_at(A.seed, key_e, (uint64_t)i, (uint64_t)c, A.cdt);
  const uint64_t ppl = pl >= 0 ? barrett64(pm * (uint64_t)pl, q, M.mu) : sub_mod(0, barrett64(pm * (uint64_t)(-pl), q, M.mu), q);
  uint64_t val = sub_mod(ppl, big_from_ntt(W2[(int64_t)blockIdx.y * n + (i - (int64_t)j * n)], qt, M), q);
  val = add_mod(val, from_signed(e, q, M.mu), q);
  Dt[c * A.R + n + i] = val;
}

// Query rows of chunk j for column c0 + y: b[t] = Delta m[c][t] - (s_j a_c)[t - j n] + e(t, c).
__global__ void k_big_emit_q(const double* W2, QEncArgs A, int64_t c0, int j, int n, uint64_t* XT, Mod M,
                             uint64_t qt, uint64_t delta, uint64_t key_e) {
  const int64_t c = c0 + blockIdx.y;
  const int64_t t = (int64_t)j * n + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.d2 || t >= (int64_t)(j + 1) * n) return;
  const uint64_t q = M.q;
  const int8_t mv = A.m_q[c * A.d2 + t];
  const uint64_t dm = mv == 1 ? delta : (mv == -1 ? (delta ? q - delta : 0) : 0);
  const int32_t e = gaussian_at(A.seed, key_e, (uint64_t)t, (uint64_t)c, A.cdt);
  uint64_t val = sub_mod(dm, big_from_ntt(W2[(int64_t)blockIdx.y * n + (t - (int64_t)j * n)], qt, M), q);
  val = add_mod(val, from_signed(e, q, M.mu), q);
  XT[c * A.K + t] = val;
}

// A-part of result column c0 + y as the NTT's doubles.
__global__ void k_big_load_col(const uint64_t* out, int64_t R_out, int64_t c0, int n, Mod M, uint64_t q, double* W) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) W[(int64_t)blockIdx.y * n + v] = big_to_ntt(out[(c0 + blockIdx.y) * R_out + v], M, q);
}

// y[c][r] = B_out[c][r] + (s'_j A_out[c])[(row0 + r) - j n] for the selected rows in chunk j.
__global__ void k_big_emit_dec(const double* W2, const uint64_t* out, int64_t R_out, int64_t row0, int64_t rows,
                               int64_t c0, int j, int n, Mod M, uint64_t qt, uint64_t* y) {
  const int64_t c = c0 + blockIdx.y;
  const int64_t lo = std::max<int64_t>((int64_t)j * n - row0, 0), hi = std::min<int64_t>((int64_t)(j + 1) * n - row0, rows);
  const int64_t r = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= hi) return;
  y[c * rows + r] = add_mod(out[c * R_out + n + r],
                            big_from_ntt(W2[(int64_t)blockIdx.y * n + (row0 + r - (int64_t)j * n)], qt, M), M.q);
}

static dim3 elem_grid(int64_t n, int64_t cols) { return dim3((unsigned)((n + 255) / 256), (unsigned)cols); }

// ------------------------------------------------------------------ launchers (same contracts as the
// LDS-resident ones in k_ntt.hip, which call these for ring degrees above 2^14)

hipError_t launch_ntt_fwd_big(uint64_t* a, int64_t count, int64_t stride, NttTab T, bool with_shoup, hipStream_t s) {
  const int n = 1 << T.logn;
  const int64_t nb = big_batch(T.logn, count);
  DevBuf W;
  hipError_t e = ws_alloc(W, sizeof(double) * nb * n, s);
  for (int64_t c0 = 0; e == hipSuccess && c0 < count; c0 += nb) {
    const int64_t cnt = std::min(nb, count - c0);
    hipLaunchKernelGGL(k_big_load_u64, elem_grid(n, cnt), dim3(256), 0, s, a + c0 * stride, stride, n, W.as<double>());
    e = hipGetLastError();
    if (e == hipSuccess) e = big_transform(W.as<double>(), cnt, T, true, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_big_store_hat, elem_grid(n, cnt), dim3(256), 0, s, W.as<double>(), n, T.q, a + c0 * stride,
                         stride, with_shoup ? 1 : 0);
      e = hipGetLastError();
    }
  }
  return e;
}

hipError_t launch_db_T_big(const int8_t* m_db, int64_t d1, int32_t d2, const uint64_t* sconj_hat, int k, NttTab T,
                           int32_t* Trow, hipStream_t s) {
  const int n = 1 << T.logn;
  const int64_t nb = big_batch(T.logn, d1);
  DevBuf W, acc;
  hipError_t e = ws_alloc(W, sizeof(double) * nb * n, s);
  if (e == hipSuccess) e = ws_alloc(acc, sizeof(double) * nb * n, s);
  for (int64_t i0 = 0; e == hipSuccess && i0 < d1; i0 += nb) {
    const int64_t cnt = std::min(nb, d1 - i0);
    for (int j = 0; e == hipSuccess && j < k; ++j) {
      hipLaunchKernelGGL(k_big_mdb_chunk, elem_grid(n, cnt), dim3(256), 0, s, m_db, d2, i0, j, n, T.qd, W.as<double>());
      e = hipGetLastError();
      if (e == hipSuccess) e = big_transform(W.as<double>(), cnt, T, true, s);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_big_pointwise, elem_grid(n, cnt), dim3(256), 0, s, W.as<double>(),
                           sconj_hat + (int64_t)j * 2 * n, n, T, acc.as<double>(), j > 0 ? 1 : 0);
        e = hipGetLastError();
      }
    }
    if (e == hipSuccess) e = big_transform(acc.as<double>(), cnt, T, false, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_big_store_T, elem_grid(n, cnt), dim3(256), 0, s, acc.as<double>(), i0, n, T.q, Trow);
      e = hipGetLastError();
    }
  }
  return e;
}

hipError_t launch_db_encrypt_big(const DbEncArgs& a, uint64_t* Dt, uint32_t prime_id, const Mod& M, NttTab T,
                                 const uint64_t* sdb_hat, hipStream_t s) {
  const int n = 1 << T.logn;
  const int64_t nb = big_batch(T.logn, a.K);
  const int chunks = (int)((a.d1 + n - 1) / n);
  DevBuf W, W2;
  hipError_t e = ws_alloc(W, sizeof(double) * nb * n, s);
  if (e == hipSuccess) e = ws_alloc(W2, sizeof(double) * nb * n, s);
  for (int64_t c0 = 0; e == hipSuccess && c0 < a.K; c0 += nb) {
    const int64_t cnt = std::min(nb, a.K - c0);
    hipLaunchKernelGGL(k_big_uniform, dim3((unsigned)((n / 4 + 255) / 256), (unsigned)cnt), dim3(256), 0, s, a.seed,
                       stream_tag(kDbA, prime_id), M, T.q, c0, n, Dt, a.R, W.as<double>());
    e = hipGetLastError();
    if (e == hipSuccess) e = big_transform(W.as<double>(), cnt, T, true, s);
    for (int j = 0; e == hipSuccess && j < chunks; ++j) {
      hipLaunchKernelGGL(k_big_pointwise, elem_grid(n, cnt), dim3(256), 0, s, W.as<double>(),
                         sdb_hat + (int64_t)j * 2 * n, n, T, W2.as<double>(), 0);
      e = hipGetLastError();
      if (e == hipSuccess) e = big_transform(W2.as<double>(), cnt, T, false, s);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_big_emit_db, elem_grid(n, cnt), dim3(256), 0, s, W2.as<double>(), a, c0, j, n, Dt, M,
                           T.q, stream_tag(kDbE, 0));
        e = hipGetLastError();
      }
    }
  }
  return e;
}

hipError_t launch_q_encrypt_big(const QEncArgs& a, uint64_t* XT, uint32_t prime_id, const Mod& M, uint64_t delta,
                                NttTab T, const uint64_t* s_hat, hipStream_t s) {
  const int n = 1 << T.logn;
  const int64_t nb = big_batch(T.logn, a.d3);
  DevBuf W, W2;
  hipError_t e = ws_alloc(W, sizeof(double) * nb * n, s);
  if (e == hipSuccess) e = ws_alloc(W2, sizeof(double) * nb * n, s);
  for (int64_t c0 = 0; e == hipSuccess && c0 < a.d3; c0 += nb) {
    const int64_t cnt = std::min(nb, a.d3 - c0);
    // a_c goes to row c of XT after the d2 b-coefficients: dst = XT + d2, stride K
    hipLaunchKernelGGL(k_big_uniform, dim3((unsigned)((n / 4 + 255) / 256), (unsigned)cnt), dim3(256), 0, s, a.seed,
                       stream_tag(kQA, prime_id), M, T.q, c0, n, XT + a.d2, a.K, W.as<double>());
    e = hipGetLastError();
    if (e == hipSuccess) e = big_transform(W.as<double>(), cnt, T, true, s);
    for (int j = 0; e == hipSuccess && j < a.k; ++j) {
      hipLaunchKernelGGL(k_big_pointwise, elem_grid(n, cnt), dim3(256), 0, s, W.as<double>(),
                         s_hat + (int64_t)j * 2 * n, n, T, W2.as<double>(), 0);
      e = hipGetLastError();
      if (e == hipSuccess) e = big_transform(W2.as<double>(), cnt, T, false, s);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_big_emit_q, elem_grid(n, cnt), dim3(256), 0, s, W2.as<double>(), a, c0, j, n, XT, M,
                           T.q, delta, stream_tag(kQE, 0));
        e = hipGetLastError();
      }
    }
  }
  return e;
}

hipError_t launch_dec_products_big(const uint64_t* out, int64_t d3, int64_t R_out, int64_t row0, int64_t rows,
                                   NttTab T, const uint64_t* sdb_hat, int j0, int j1, const Mod& M, uint64_t* y,
                                   hipStream_t s) {
  const int n = 1 << T.logn;
  const int64_t nb = big_batch(T.logn, d3);
  DevBuf W, W2;
  hipError_t e = ws_alloc(W, sizeof(double) * nb * n, s);
  if (e == hipSuccess) e = ws_alloc(W2, sizeof(double) * nb * n, s);
  for (int64_t c0 = 0; e == hipSuccess && c0 < d3; c0 += nb) {
    const int64_t cnt = std::min(nb, d3 - c0);
    hipLaunchKernelGGL(k_big_load_col, elem_grid(n, cnt), dim3(256), 0, s, out, R_out, c0, n, M, T.q, W.as<double>());
    e = hipGetLastError();
    if (e == hipSuccess) e = big_transform(W.as<double>(), cnt, T, true, s);
    for (int j = j0; e == hipSuccess && j <= j1; ++j) {
      hipLaunchKernelGGL(k_big_pointwise, elem_grid(n, cnt), dim3(256), 0, s, W.as<double>(),
                         sdb_hat + (int64_t)j * 2 * n, n, T, W2.as<double>(), 0);
      e = hipGetLastError();
      if (e == hipSuccess) e = big_transform(W2.as<double>(), cnt, T, false, s);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_big_emit_dec, elem_grid(n, cnt), dim3(256), 0, s, W2.as<double>(), out, R_out, row0,
                           rows, c0, j, n, M, T.q, y);
        e = hipGetLastError();
      }
    }
  }
  return e;
}

}  // namespace hfe
