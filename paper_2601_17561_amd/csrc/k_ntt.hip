// Negacyclic NTT (LDS-resident, ring degrees up to 2^14) and the kernels built on it:
// secret-key transforms, T = M_DB S_Q, database and query encryption, decryption products.
// Larger ring degrees (2^15, 2^16) go through the two-pass transforms of k_ntt_big.hip, which the
// launchers below call with the same arguments.
//
// Products in R_n = Z[X]/(X^n + 1) mod a 36-bit prime q (Section 2.2.1) are computed as
// INTT(NTT(a) . NTT(s)) with the merged negacyclic transforms of Longa and Naehrig (2016):
// forward Cooley-Tukey with twiddles psi^brv(i) (output in bit-reversed order), inverse
// Gentleman-Sande with psi^-brv(i) and a final 1/n scale.  One workgroup transforms one
// polynomial held in LDS (2^14 x 8 bytes = 128 KiB fits the 160 KiB LDS of a gfx950 CU).
// Inside the transforms residues are held as doubles (exact integers below 2^36) and multiplied
// mod q with an error-free fp64 product (see mulmod_d): about a third of the integer instructions
// of a 64-bit Shoup product, at the same issue rate on this chip.
#include <type_traits>

#include "hfe_ntt_lds.h"

namespace hfe {

// The n^2 modulus chain multiplies by the ternary secrets through the NTT prime q of the tables: a
// residue x mod m (m = n^2 < 2^16) enters as its centered integer taken mod q, and every product
// coefficient is an integer of magnitude at most N m / 2 <= 2^31 < q / 2, so the centered result mod
// q is that integer, which is then reduced mod m.  (For the 36-bit primes m = q and neither step
// runs.)
__device__ __forceinline__ double to_ntt(uint64_t x, uint64_t m, uint64_t q) {
  const int64_t c = centered(x, m);
  return (double)(c >= 0 ? (uint64_t)c : q - (uint64_t)(-c));
}
__device__ __forceinline__ uint64_t from_ntt(double v, uint64_t q, const Mod& M) {
  return from_signed(centered((uint64_t)v, q), M.q, M.mu);
}

// ------------------------------------------------------------------ batch forward NTT

__global__ void __launch_bounds__(kNttThreads) k_ntt_fwd(uint64_t* a, int64_t stride, NttTab T,
                                                          int with_shoup) {
  extern __shared__ double lds[];
  const int n = 1 << T.logn;
  uint64_t* poly = a + (int64_t)blockIdx.x * stride;
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = to_d(poly[i]);
  __syncthreads();
  ntt_fwd_lds(lds, T);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint64_t v = to_u(lds[i]);
    poly[i] = v;
    if (with_shoup) poly[n + i] = shoup_quot(v, T.q);
  }
}

hipError_t launch_ntt_fwd(uint64_t* a, int64_t count, int64_t stride, NttTab tab, bool with_shoup,
                          hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (tab.logn > kMaxLogN) return launch_ntt_fwd_big(a, count, stride, tab, with_shoup, s);
  const size_t lds = sizeof(double) << tab.logn;
  hipError_t e = allow_lds(k_ntt_fwd, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ntt_fwd, dim3((unsigned)count), dim3(ntt_block(tab.logn)), lds, s, a, stride, tab,
                     with_shoup ? 1 : 0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ T = M_DB S_Q
// Row i of T is sum_j s~_j * m_i^(j) in R_{N_Q} (s~_j(X) = s_j(1/X), m_i^(j) = chunk j of
// row i).  Exact integers with |T| <= d2 < q_0 / 2, so one prime suffices; the sum is
// accumulated in the NTT domain in registers.  Output row-major T[i][v] (int32).


template <int R>
__global__ void __launch_bounds__(kNttThreads)
k_db_T(const int8_t* m_db, int32_t d2, const uint64_t* sconj_hat, int k, NttTab T, int32_t* Trow) {
  extern __shared__ double lds[];
  const int n = 1 << T.logn;
  const int64_t i = blockIdx.x;
  const double q = T.qd, qinv = T.qinv;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int j = 0; j < k; ++j) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      const int64_t col = (int64_t)j * n + t;
      const int8_t m = col < d2 ? m_db[i * d2 + col] : (int8_t)0;
      lds[t] = m == 1 ? 1.0 : (m == -1 ? q - 1.0 : 0.0);
    }
    __syncthreads();
    ntt_fwd_lds(lds, T);
    const uint64_t* w = sconj_hat + (int64_t)j * 2 * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = threadIdx.x + r * blockDim.x;
      if (t < n) acc[r] = addmod_d(acc[r], mulmod_d(lds[t], to_d(w[t]), q, qinv), q);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = threadIdx.x + r * blockDim.x;
    if (t < n) lds[t] = acc[r];
  }
  __syncthreads();
  ntt_inv_lds(lds, T);
  for (int t = threadIdx.x; t < n; t += blockDim.x) Trow[i * n + t] = (int32_t)centered(to_u(lds[t]), T.q);
}

__global__ void k_transpose_i32(const int32_t* in, int64_t rows, int64_t cols, int32_t* out) {
  __shared__ int32_t tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int64_t r = r0 + y, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[y][threadIdx.x] = in[r * cols + c];
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int64_t c = c0 + y, r = r0 + threadIdx.x;
    if (r < rows && c < cols) out[c * rows + r] = tile[threadIdx.x][y];
  }
}

hipError_t launch_db_T(const int8_t* m_db, int64_t d1, int32_t d2, const uint64_t* sconj_hat, int k,
                       NttTab tab_q0, int32_t* Trow, int32_t* Tt, hipStream_t s) {
  if (d1 <= 0) return hipSuccess;
  const int n = 1 << tab_q0.logn;
  const size_t lds = sizeof(double) * n;
  hipError_t e = tab_q0.logn > kMaxLogN ? launch_db_T_big(m_db, d1, d2, sconj_hat, k, tab_q0, Trow, s)
                                        : by_regs(regs_per_thread(tab_q0.logn), [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    hipError_t e2 = allow_lds(k_db_T<R>, lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL(k_db_T<R>, dim3((unsigned)d1), dim3(ntt_block(tab_q0.logn)), lds, s, m_db, d2,
                       sconj_hat, k, tab_q0, Trow);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((d1 + 31) / 32));
  hipLaunchKernelGGL(k_transpose_i32, grid, dim3(32, 8), 0, s, Trow, d1, (int64_t)n, Tt);
  return hipGetLastError();
}

// ------------------------------------------------------------------ database encryption
// One workgroup per column c of D (one a-polynomial): a_c uniform (stream DBA, element
// (v, c)), then for each database chunk j the product s'_j * a_c, and for database rows i of
// chunk j: B[i][c] = -(s'_j a_c)[i - j N_DB] + p * plain[i][c] + e(i, c) (stream DBE).
// plain = M_DB for c < d2, T for c >= d2.  Column c of D is stored contiguously: Dt[c][row].

template <int R, bool CHAIN>
__global__ void __launch_bounds__(kNttThreads)
k_db_encrypt(DbEncArgs A, uint64_t* Dt, uint32_t prime_id, Mod M, NttTab T, const uint64_t* sdb_hat) {
  extern __shared__ double lds[];
  const int n = 1 << T.logn;
  const int64_t c = blockIdx.x;
  const uint64_t q = M.q;
  uint64_t* col = Dt + c * A.R;
  const uint64_t key_a = stream_tag(kDbA, prime_id);
  for (int v4 = threadIdx.x; v4 < (n + 3) / 4; v4 += blockDim.x) {
    const Philox4 b = philox4x64_10(A.seed, key_a, (uint64_t)v4, (uint64_t)c, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int v = 4 * v4 + j;
      if (v < n) {
        const uint64_t w = b.v[j];
        const uint64_t x = w < M.bound ? barrett64(w, q, M.mu)
                                       : uniform_at(A.seed, key_a, (uint64_t)v, (uint64_t)c, M);
        lds[v] = CHAIN ? to_ntt(x, q, T.q) : to_d(x);
        col[v] = x;
      }
    }
  }
  __syncthreads();
  // NTT(a_c) once, kept in registers for all chunks.
  ntt_fwd_lds(lds, T);
  double ahat[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int v = threadIdx.x + r * blockDim.x;
    ahat[r] = v < n ? lds[v] : 0.0;
  }
  const uint64_t pm = barrett64(A.p, q, M.mu);
  const uint64_t key_e = stream_tag(kDbE, 0);
  const int chunks = (int)((A.d1 + n - 1) / n);
  for (int j = 0; j < chunks; ++j) {
    const uint64_t* w = sdb_hat + (int64_t)j * 2 * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int v = threadIdx.x + r * blockDim.x;
      if (v < n) lds[v] = mulmod_d(ahat[r], to_d(w[v]), T.qd, T.qinv);
    }
    __syncthreads();
    ntt_inv_lds(lds, T);
    const int64_t lo = (int64_t)j * n;
    const int64_t hi = lo + n < A.d1 ? lo + n : A.d1;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const int32_t pl = c < A.d2 ? (int32_t)A.MT[c * A.d1 + i] : A.Tt[(c - A.d2) * A.d1 + i];
      const int32_t e = gaussian_at(A.seed, key_e, (uint64_t)i, (uint64_t)c, A.cdt);
      const uint64_t ppl = pl >= 0 ? barrett64(pm * (uint64_t)pl, q, M.mu)
                                   : sub_mod(0, barrett64(pm * (uint64_t)(-pl), q, M.mu), q);
      uint64_t val = sub_mod(ppl, CHAIN ? from_ntt(lds[i - lo], T.q, M) : to_u(lds[i - lo]), q);
      val = add_mod(val, from_signed(e, q, M.mu), q);
      col[n + i] = val;
    }
    __syncthreads();
  }
}

hipError_t launch_db_encrypt(const DbEncArgs& a, uint64_t* Dt_prime, uint32_t prime_id, const Mod& m,
                             NttTab tab_db, const uint64_t* sdb_hat_prime, hipStream_t s) {
  if (a.K <= 0) return hipSuccess;
  if (tab_db.logn > kMaxLogN) return launch_db_encrypt_big(a, Dt_prime, prime_id, m, tab_db, sdb_hat_prime, s);
  const size_t lds = sizeof(double) << tab_db.logn;
  const bool chain = m.q != tab_db.q;  // residues mod n^2, products through the table's prime
  return by_regs(regs_per_thread(tab_db.logn), [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    auto kern = chain ? k_db_encrypt<R, true> : k_db_encrypt<R, false>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)a.K), dim3(ntt_block(tab_db.logn)), lds, s, a, Dt_prime, prime_id, m,
                       tab_db, sdb_hat_prime);
    return hipGetLastError();
  });
}

// ------------------------------------------------------------------ query encryption
// One workgroup per query column c: a_c uniform in R_{N_Q} (stream QA, element (t, c)), and
// for each chunk j of N_Q code rows b[t] = -(s_j a_c)[t - j N_Q] + Delta m[c][t] + e(t, c).
// Output row c of XT: [b_c (d2) | a_c (N_Q)].

template <int R, bool CHAIN>
__global__ void __launch_bounds__(kNttThreads)
k_q_encrypt(QEncArgs A, uint64_t* XT, uint32_t prime_id, Mod M, uint64_t delta, NttTab T,
            const uint64_t* s_hat) {
  extern __shared__ double lds[];
  const int n = 1 << T.logn;
  const int64_t c = blockIdx.x;
  const uint64_t q = M.q;
  uint64_t* row = XT + c * A.K;
  uint64_t* arow = row + A.d2;
  const uint64_t key_a = stream_tag(kQA, prime_id);
  for (int t4 = threadIdx.x; t4 < (n + 3) / 4; t4 += blockDim.x) {
    const Philox4 b = philox4x64_10(A.seed, key_a, (uint64_t)t4, (uint64_t)c, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = 4 * t4 + j;
      if (t < n) {
        const uint64_t w = b.v[j];
        const uint64_t x = w < M.bound ? barrett64(w, q, M.mu)
                                       : uniform_at(A.seed, key_a, (uint64_t)t, (uint64_t)c, M);
        lds[t] = CHAIN ? to_ntt(x, q, T.q) : to_d(x);
        arow[t] = x;
      }
    }
  }
  __syncthreads();
  // NTT(a_c) once (signed, uncorrected: below 8.1q), kept in registers (n / blockDim = R values per
  // thread) for all chunks.
  ntt_fwd_lds_c(lds, T);
  double ahat[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = threadIdx.x + r * blockDim.x;
    ahat[r] = t < n ? lds[t] : 0.0;
  }
  const uint64_t key_e = stream_tag(kQE, 0);
  const int8_t* m = A.m_q + c * A.d2;
  for (int j = 0; j < A.k; ++j) {
    const uint64_t* w = s_hat + (int64_t)j * 2 * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = threadIdx.x + r * blockDim.x;
      if (t < n) lds[t] = mulmod_c_d(ahat[r], to_d(w[t]), T.qd, T.qinv);  // centered
    }
    __syncthreads();
    ntt_inv_lds_c(lds, T);  // residues in [0, q)
    const int64_t lo = (int64_t)j * n;
    const int64_t hi = lo + n < A.d2 ? lo + n : A.d2;
    // positions in pairs (lo is even): the errors drawn once for every prime, or both Gaussians of a
    // pair from one Philox block
    for (int64_t t = lo + 2 * (int64_t)threadIdx.x; t < hi; t += 2 * (int64_t)blockDim.x) {
      int32_t e2[2];
      if (A.e) {
        e2[0] = A.e[c * A.d2 + t];
        e2[1] = t + 1 < hi ? A.e[c * A.d2 + t + 1] : 0;
      } else {
        gaussian_pair_at(A.seed, key_e, (uint64_t)t >> 1, (uint64_t)c, A.cdt, e2[0], e2[1]);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (t + h >= hi) break;
        const int8_t mv = m[t + h];
        const uint64_t dm = mv == 1 ? delta : (mv == -1 ? (delta ? q - delta : 0) : 0);
        uint64_t val = sub_mod(dm, CHAIN ? from_ntt(lds[t + h - lo], T.q, M) : to_u(lds[t + h - lo]), q);
        val = add_mod(val, from_signed(e2[h], q, M.mu), q);
        row[t + h] = val;
      }
    }
    __syncthreads();
  }
}

__global__ void k_q_errors(uint64_t seed, const uint64_t* cdt, int64_t d3, int64_t d2, int8_t* e) {
  const int64_t half = (d2 + 1) / 2, n = d3 * half;
  const uint64_t key_e = stream_tag(kQE, 0);
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = x / half, u = x - c * half;
    int32_t e0, e1;
    gaussian_pair_at(seed, key_e, (uint64_t)u, (uint64_t)c, cdt, e0, e1);
    e[c * d2 + 2 * u] = (int8_t)e0;
    if (2 * u + 1 < d2) e[c * d2 + 2 * u + 1] = (int8_t)e1;
  }
}

hipError_t launch_q_errors(uint64_t seed, const uint64_t* cdt, int64_t d3, int64_t d2, int8_t* e, hipStream_t s) {
  const int64_t n = d3 * ((d2 + 1) / 2);
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_q_errors, dim3((unsigned)blocks), dim3(256), 0, s, seed, cdt, d3, d2, e);
  return hipGetLastError();
}

hipError_t launch_q_encrypt(const QEncArgs& a, uint64_t* XT_prime, uint32_t prime_id, const Mod& m,
                            uint64_t delta_mod, NttTab tab_q, const uint64_t* s_hat_prime,
                            hipStream_t s) {
  if (a.d3 <= 0) return hipSuccess;
  if (tab_q.logn > kMaxLogN) return launch_q_encrypt_big(a, XT_prime, prime_id, m, delta_mod, tab_q, s_hat_prime, s);
  const size_t lds = sizeof(double) << tab_q.logn;
  const bool chain = m.q != tab_q.q;  // residues mod n^2, products through the table's prime
  return by_regs(regs_per_thread(tab_q.logn), [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    auto kern = chain ? k_q_encrypt<R, true> : k_q_encrypt<R, false>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)a.d3), dim3(ntt_block(tab_q.logn)), lds, s, a, XT_prime, prime_id, m,
                       delta_mod, tab_q, s_hat_prime);
    return hipGetLastError();
  });
}

// ------------------------------------------------------------------ decryption products
// Workgroup (c, j): y[c][r] = B_out[c][r] + (s'_j * A_out[c])[(row0 + r) - j N_DB] for the
// selected rows r whose database row row0 + r lies in chunk j.

template <bool CHAIN>
__global__ void __launch_bounds__(kNttThreads)
k_dec_products(const uint64_t* out, int64_t R_out, int64_t row0, int64_t rows, NttTab T,
               const uint64_t* sdb_hat, int j0, Mod M, uint64_t* y) {
  extern __shared__ double lds[];
  const int n = 1 << T.logn;
  const int64_t c = blockIdx.x;
  const int j = j0 + (int)blockIdx.y;
  const uint64_t q = M.q;  // the arithmetic modulus (the table's prime, or n^2 of the chain)
  const uint64_t* ocol = out + c * R_out;
  // loads staged four per thread (all issued before the first is used)
  staged_pass<4>(n, [&](int v) { return ocol[v]; },
                 [&](int v, uint64_t x) { lds[v] = CHAIN ? to_ntt(x, q, T.q) : to_d(x); });
  __syncthreads();
  ntt_fwd_lds_c(lds, T);  // signed, uncorrected: below 8.1q
  const uint64_t* w = sdb_hat + (int64_t)j * 2 * n;
  staged_pass<4>(n, [&](int v) { return w[v]; },
                 [&](int v, uint64_t x) { lds[v] = mulmod_c_d(lds[v], to_d(x), T.qd, T.qinv); });
  __syncthreads();
  ntt_inv_lds_c(lds, T);  // residues in [0, q)
  int64_t lo = (int64_t)j * n - row0, hi = lo + n;
  if (lo < 0) lo = 0;
  if (hi > rows) hi = rows;
  staged_range<4>(lo, hi, [&](int64_t r) { return ocol[n + r]; }, [&](int64_t r, uint64_t b) {
    y[c * rows + r] = add_mod(b, CHAIN ? from_ntt(lds[row0 + r - (int64_t)j * n], T.q, M)
                                       : to_u(lds[row0 + r - (int64_t)j * n]), q);
  });
}

hipError_t launch_dec_products(const uint64_t* out_prime, int64_t d3, int64_t R_out, int64_t row0,
                               int64_t rows, int n_db_log, NttTab tab, const uint64_t* sdb_hat_prime,
                               int k_db, uint64_t* y_prime, hipStream_t s, const Mod* arith) {
  if (d3 <= 0 || rows <= 0) return hipSuccess;
  const int64_t n = 1ll << n_db_log;
  const int j0 = (int)(row0 / n), j1 = (int)((row0 + rows - 1) / n);
  if (j1 >= k_db) return hipErrorInvalidValue;
  Mod M;
  M.q = tab.q;
  M.mu = 0;
  M.bound = 0;
  if (arith) M = *arith;
  const bool chain = M.q != tab.q;
  if (tab.logn > kMaxLogN)
    return launch_dec_products_big(out_prime, d3, R_out, row0, rows, tab, sdb_hat_prime, j0, j1, M, y_prime, s);
  const size_t lds = sizeof(double) << tab.logn;
  auto kern = chain ? k_dec_products<true> : k_dec_products<false>;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)d3, (unsigned)(j1 - j0 + 1)), dim3(ntt_block(tab.logn)), lds, s, out_prime,
                     R_out, row0, rows, tab, sdb_hat_prime, j0, M, y_prime);
  return hipGetLastError();
}

}  // namespace hfe
