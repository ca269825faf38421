// FormatSwitch (Appendix C.1): the query from its transmission ring R_{N_T} to the MSRLWE format of
// the CCMM in R_{N_Q}, and the client's transmission encryption that produces its input.
//
// A transmission ciphertext (a, b) mod Q' = q_0 .. q_l in R_{N_T} holds one chunk of N_Q code
// positions of a query column at the coefficients of degree divisible by rho = N_T / N_Q.  The switch
// key-switches a from s_T to s'(X^rho) (one digit per prime of Q', keys mod Q' p, RS_p) and keeps the
// coefficients of degree divisible by rho (the trace), converts the k chunks of a column to one MSRLWE
// ciphertext under the CCMM secrets s_0 .. s_{k-1} (conversion keys with a shared mask per digit and
// chunk, RS_p), and switches the modulus from Q' to Q_l = q_0 .. q_{l-1} (RS_{q_l}).
//
// The trace is taken without any transform of degree N_T.  Write f(X) = sum_{r < rho} X^r f_r(X^rho)
// for f in R_{N_T} (its polyphase parts, polynomials in Y = X^rho, Y^{N_Q} = -1).  The part of degree
// divisible by rho of a product d K is d_0 K_0 + Y sum_{r >= 1} d_r K_{rho - r}, so the switched
// mask and key parts are sums over the digits i and the parts r of products in R_{N_Q}.  The keys are
// stored as the transforms of K~_0 = K_0 and K~_r = Y K_{rho - r}; each product is then one
// LDS-resident NTT of d_r per (digit, part, slot) and a pointwise multiply-accumulate held in
// registers, and one inverse transform per result.  Every value is the exact residue that the full
// key switch followed by the extraction gives.
#include "hfe_ntt_lds.h"

namespace hfe {

// Rescale of one coefficient by the modulus D: (x_q - [x_D]) D^-1 mod q, with [x_D] the centered
// residue in (-D/2, D/2) and dinv = D^-1 mod q.  x_q - [x_D] lies in (-D/2, q + D/2), and D < 2q, so
// one correction each way brings it to [0, q).
__device__ __forceinline__ double rs_d(double xq, double xD, double D, double q, double qinv, double dinv) {
  const double c = xD > 0.5 * D ? xD - D : xD;
  double d = xq - c;
  d = d < 0.0 ? d + q : (d >= q ? d - q : d);
  return mulmod_d(d, dinv, q, qinv);
}

// Flat work index of workgroup b for a grid of G items spread over the 8 XCDs in contiguous runs:
// the hardware places workgroup b on XCD b mod 8, so consecutive items (the slots of one column) run
// together on one XCD and share its L2 for the column's digits.
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t G) {
  const int64_t per = (G + 7) / 8;
  return (b & 7) * per + (b >> 3);
}
static unsigned xcd_grid(int64_t G) { return (unsigned)(((G + 7) / 8) * 8); }

// ------------------------------------------------------------------ ring-switching keys
// Coefficients of K~_r for slot z, digit i: the mask k_i (stream RkA of slot z, element (t, i)) and
// g_i s_T + e_i (stream RkE, element (t, i)) at t = rho u' + src, src = 0 for r = 0 and rho - r
// otherwise, u' = u for r = 0 and u - 1 otherwise (the product by Y: coefficient u - 1 moves to u and
// coefficient N_Q - 1 wraps to 0 with its sign flipped).
__global__ void k_fs_rk_coeffs(FsConsts C, uint64_t seed, const int8_t* st, const uint64_t* cdt, uint64_t* out) {
  const int nq = 1 << C.logn_q;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nq) return;
  const int r = blockIdx.y;
  const int zi = blockIdx.z;
  const int z = zi / (C.level + 1), i = zi - z * (C.level + 1);
  const int src = r ? C.rho - r : 0;
  int uu = u;
  bool neg = false;
  if (r) {
    neg = u == 0;
    uu = neg ? nq - 1 : u - 1;
  }
  const uint64_t t = (uint64_t)C.rho * (uint64_t)uu + (uint64_t)src;
  const Mod& M = C.mod[z];
  uint64_t a = uniform_at(seed, stream_tag(kRkA, C.pid[z]), t, (uint64_t)i, M);
  const int32_t e = gaussian_at(seed, stream_tag(kRkE, 0), t, (uint64_t)i, cdt);
  uint64_t b = from_signed(e, M.q, M.mu);
  const int sv = st[t];
  if (sv == 1) b = add_mod(b, C.gk[z][i], M.q);
  if (sv == -1) b = sub_mod(b, C.gk[z][i], M.q);
  if (neg) {
    a = a ? M.q - a : 0;
    b = b ? M.q - b : 0;
  }
  const size_t base = (size_t)zi * 2 * C.rho * nq;
  out[base + (size_t)r * nq + u] = a;
  out[base + (size_t)(C.rho + r) * nq + u] = b;
}

hipError_t launch_fs_rk_coeffs(const FsConsts& C, uint64_t seed, const int8_t* st, const uint64_t* cdt,
                               uint64_t* out, hipStream_t s) {
  const int nq = 1 << C.logn_q;
  dim3 grid((unsigned)((nq + 255) / 256), (unsigned)C.rho, (unsigned)(C.nz * (C.level + 1)));
  hipLaunchKernelGGL(k_fs_rk_coeffs, grid, dim3(256), 0, s, C, seed, st, cdt, out);
  return hipGetLastError();
}

// rk[z][i][0][r] = NTT(K~ mask), rk[z][i][1][r] = NTT(K~ key) = NTT(g s_T + e part) - NTT(s') NTT(mask)
// (the key is -k_i s'(X^rho) + g_i s_T + e_i, and s'(X^rho) has only the polyphase part 0, s').
__global__ void k_fs_rk_finish(FsConsts C, const uint64_t* coef_hat, const uint64_t* sr_hat, double* rk) {
  const int nq = 1 << C.logn_q;
  const int64_t per_zi = (int64_t)C.rho * nq;
  const int64_t n = (int64_t)C.nz * (C.level + 1) * per_zi;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t zi = x / per_zi, w = x - zi * per_zi;
    const int z = (int)(zi / (C.level + 1));
    const int v = (int)(w % nq);
    const size_t ia = (size_t)zi * 2 * per_zi + w, ib = ia + per_zi;
    const double q = C.zd[z], qinv = C.zinv[z];
    const double a = to_d(coef_hat[ia]);
    const double sa = mulmod_d(to_d(sr_hat[(size_t)z * nq + v]), a, q, qinv);
    rk[ia] = a;
    rk[ib] = submod_d(to_d(coef_hat[ib]), sa, q);
  }
}

hipError_t launch_fs_rk_finish(const FsConsts& C, const uint64_t* coef_hat, const uint64_t* sr_hat, double* rk,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_fs_rk_finish, dim3(2048), dim3(256), 0, s, C, coef_hat, sr_hat, rk);
  return hipGetLastError();
}

// ------------------------------------------------------------------ conversion keys
// For slot z, digit i, input chunk j (idx = i k + j): the shared mask k_ij (stream CkA of slot z,
// element (u, idx)) and, per output j', e (stream CkE, element (u, idx k + j')) plus g_i s' when j' = j.
__global__ void k_fs_ck_coeffs(FsConsts C, uint64_t seed, const int8_t* sr, const uint64_t* cdt, uint64_t* out) {
  const int nq = 1 << C.logn_q;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nq) return;
  const int idx = blockIdx.y;  // i k + j
  const int z = blockIdx.z;
  const int i = idx / C.k, j = idx - i * C.k;
  const Mod& M = C.mod[z];
  uint64_t* o = out + ((size_t)z * (C.level + 1) * C.k + idx) * (1 + C.k) * nq;
  o[u] = uniform_at(seed, stream_tag(kCkA, C.pid[z]), (uint64_t)u, (uint64_t)idx, M);
  const int sv = sr[u];
  for (int jp = 0; jp < C.k; ++jp) {
    const int32_t e = gaussian_at(seed, stream_tag(kCkE, 0), (uint64_t)u, (uint64_t)(idx * C.k + jp), cdt);
    uint64_t b = from_signed(e, M.q, M.mu);
    if (jp == j && sv == 1) b = add_mod(b, C.gk[z][i], M.q);
    if (jp == j && sv == -1) b = sub_mod(b, C.gk[z][i], M.q);
    o[(size_t)(1 + jp) * nq + u] = b;
  }
}

hipError_t launch_fs_ck_coeffs(const FsConsts& C, uint64_t seed, const int8_t* sr, const uint64_t* cdt,
                               uint64_t* out, hipStream_t s) {
  const int nq = 1 << C.logn_q;
  dim3 grid((unsigned)((nq + 255) / 256), (unsigned)((C.level + 1) * C.k), (unsigned)C.nz);
  hipLaunchKernelGGL(k_fs_ck_coeffs, grid, dim3(256), 0, s, C, seed, sr, cdt, out);
  return hipGetLastError();
}

// ck[z][i][j][0] = NTT(k_ij); ck[z][i][j][1 + j'] = NTT(e part) - NTT(s_j') NTT(k_ij).
__global__ void k_fs_ck_finish(FsConsts C, const uint64_t* coef_hat, const uint64_t* s_hat, int p_index,
                               double* ck) {
  const int nq = 1 << C.logn_q;
  const int64_t per = (int64_t)(1 + C.k) * nq;
  const int64_t n = (int64_t)C.nz * (C.level + 1) * C.k * per;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = x / per, w = x - blk * per;
    const int z = (int)(blk / ((C.level + 1) * C.k));
    const int part = (int)(w / nq), v = (int)(w - (int64_t)part * nq);
    const double q = C.zd[z], qinv = C.zinv[z];
    const double a = to_d(coef_hat[(size_t)blk * per + v]);
    if (part == 0) {
      ck[x] = a;
    } else {
      const int slot = z <= C.level ? z : p_index;
      const uint64_t* sh = s_hat + ((size_t)slot * C.k + (part - 1)) * 2 * nq;
      ck[x] = submod_d(to_d(coef_hat[x]), mulmod_d(to_d(sh[v]), a, q, qinv), q);
    }
  }
}

hipError_t launch_fs_ck_finish(const FsConsts& C, const uint64_t* coef_hat, const uint64_t* s_hat, int p_index,
                               double* ck, hipStream_t s) {
  hipLaunchKernelGGL(k_fs_ck_finish, dim3(1024), dim3(256), 0, s, C, coef_hat, s_hat, p_index, ck);
  return hipGetLastError();
}

// ------------------------------------------------------------------ transmission encryption
// Ciphertext col = c k + j, prime i <= l: a uniform (stream TxA of prime i, element (t, col)),
// b = -s_T a + (Delta_l q_l) m~ + e (stream TxE, element (t, col)), m~ holding positions
// [j N_Q, (j + 1) N_Q) of query column c at the coefficients rho u.  s_T a is taken part by part:
// part c' of the product is sum_{r <= c'} S_r A_{c'-r} + Y sum_{r > c'} S_r A_{c'+rho-r}.
// T layout: [i <= l][col][a | b][N_T].

// Workgroup (col, i rho + r): draws part r of a, writes its coefficients to T, and its transform.
__global__ void __launch_bounds__(kNttThreads)
k_fs_tx_a(FsConsts C, uint64_t seed, int64_t ncols, double* Ahat, uint64_t* T) {
  extern __shared__ double lds[];
  const int nq = 1 << C.logn_q;
  const int64_t nt = (int64_t)nq * C.rho;
  const int64_t col = blockIdx.x;
  const int i = blockIdx.y / C.rho, r = blockIdx.y - i * C.rho;
  const Mod& M = C.mod[i];
  uint64_t* a = T + ((size_t)i * ncols + col) * 2 * nt;
  for (int u = threadIdx.x; u < nq; u += blockDim.x) {
    const uint64_t t = (uint64_t)C.rho * u + r;
    const uint64_t x = uniform_at(seed, stream_tag(kTxA, (uint64_t)i), t, (uint64_t)col, M);
    a[t] = x;
    lds[u] = to_d(x);
  }
  __syncthreads();
  ntt_fwd_lds(lds, C.tab[i]);
  double* o = Ahat + (((size_t)col * (C.level + 1) + i) * C.rho + r) * nq;
  for (int v = threadIdx.x; v < nq; v += blockDim.x) o[v] = lds[v];
}

// Workgroup (col, i rho + c'): part c' of s_T a, then b at the coefficients rho u + c'.
template <int R>
__global__ void __launch_bounds__(kNttThreads)
k_fs_tx_b(FsConsts C, uint64_t seed, const int8_t* m_q, int64_t ncols, const uint64_t* st_hat,
          const uint64_t* y_hat, const uint64_t* cdt, const double* Ahat, uint64_t* T) {
  extern __shared__ double lds[];
  const int nq = 1 << C.logn_q;
  const int64_t nt = (int64_t)nq * C.rho;
  const int64_t col = blockIdx.x;
  const int i = blockIdx.y / C.rho, cp = blockIdx.y - i * C.rho;
  const double q = C.zd[i], qinv = C.zinv[i];
  const double* A = Ahat + ((size_t)col * (C.level + 1) + i) * C.rho * nq;
  const uint64_t* S = st_hat + (size_t)i * C.rho * nq;
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int v = threadIdx.x + k * blockDim.x;
    double lo = 0.0, hi = 0.0;
    for (int r = 0; r < C.rho; ++r) {
      const bool wrap = r > cp;
      const int src = wrap ? cp + C.rho - r : cp - r;
      const double pr = mulmod_d(to_d(S[(size_t)r * nq + v]), A[(size_t)src * nq + v], q, qinv);
      if (wrap)
        hi = addmod_d(hi, pr, q);
      else
        lo = addmod_d(lo, pr, q);
    }
    acc[k] = addmod_d(lo, mulmod_d(hi, to_d(y_hat[(size_t)i * nq + v]), q, qinv), q);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) lds[threadIdx.x + k * blockDim.x] = acc[k];
  __syncthreads();
  ntt_inv_lds_c(lds, C.tab[i]);
  const int64_t c = col / C.k, j = col - c * C.k;
  const Mod& M = C.mod[i];
  const uint64_t sc = (uint64_t)C.scale[i];
  uint64_t* b = T + (((size_t)i * ncols + col) * 2 + 1) * nt;
  for (int u = threadIdx.x; u < nq; u += blockDim.x) {
    const uint64_t t = (uint64_t)C.rho * u + cp;
    const int64_t pos = j * nq + u;
    const int mv = (cp == 0 && pos < C.d2) ? (int)m_q[c * C.d2 + pos] : 0;
    const int32_t e = gaussian_at(seed, stream_tag(kTxE, 0), t, (uint64_t)col, cdt);
    uint64_t val = sub_mod(from_signed(e, M.q, M.mu), to_u(lds[u]), M.q);
    if (mv == 1) val = add_mod(val, sc, M.q);
    if (mv == -1) val = sub_mod(val, sc, M.q);
    b[t] = val;
  }
}

hipError_t launch_fs_tx(const FsConsts& C, uint64_t seed, const int8_t* m_q, int64_t d3, const uint64_t* st_hat,
                        const uint64_t* y_hat, const uint64_t* cdt, double* Ahat, uint64_t* T, hipStream_t s) {
  const int64_t ncols = d3 * C.k;
  if (ncols <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn_q;
  const dim3 grid((unsigned)ncols, (unsigned)((C.level + 1) * C.rho));
  return by_regs(regs_per_thread(C.logn_q), [&](auto rc) -> hipError_t {
    constexpr int R = decltype(rc)::value;
    hipError_t e = allow_lds(k_fs_tx_a, lds);
    if (e == hipSuccess) e = allow_lds(k_fs_tx_b<R>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fs_tx_a, grid, dim3(ntt_block(C.logn_q)), lds, s, C, seed, ncols, Ahat, T);
    hipLaunchKernelGGL(k_fs_tx_b<R>, grid, dim3(ntt_block(C.logn_q)), lds, s, C, seed, m_q, ncols, st_hat, y_hat,
                       cdt, Ahat, T);
    return hipGetLastError();
  });
}

// ------------------------------------------------------------------ the switch
// Digits d_i = [a (Q'/q_i)^-1]_{q_i} of every mask a, in polyphase order: Dg[col][i][r][u] is the
// digit of coefficient rho u + r.
__global__ void k_fs_digits(FsConsts C, const uint64_t* T, int64_t ncols, double* Dg) {
  const int nq = 1 << C.logn_q;
  const int64_t nt = (int64_t)nq * C.rho;
  const int64_t col = blockIdx.x / (C.level + 1);
  const int i = (int)(blockIdx.x - col * (C.level + 1));
  const double q = C.zd[i], qinv = C.zinv[i], g = C.ghat[i];
  const uint64_t* a = T + ((size_t)i * ncols + col) * 2 * nt;
  double* o = Dg + ((size_t)col * (C.level + 1) + i) * nt;
  // thread u takes the rho coefficients u rho .. u rho + rho - 1 (contiguous across the wavefront) and writes
  // part r at r N_Q + u (consecutive u across the wavefront): both sides coalesced
  if (C.rho == 8) {
    for (int u = threadIdx.x; u < nq; u += blockDim.x) {
      const uint64_t* src = a + (int64_t)u * 8;
      uint64_t x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = src[r];
#pragma unroll
      for (int r = 0; r < 8; ++r) o[(int64_t)r * nq + u] = mulmod_d(to_d(x[r]), g, q, qinv);
    }
    return;
  }
  for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) {
    const int64_t u = t / C.rho, r = t - u * C.rho;
    o[r * nq + u] = mulmod_d(to_d(a[t]), g, q, qinv);
  }
}

// The forward transforms are fused with their load and their use (ntt_fwd_fused, hfe_ntt_lds.h).

// acc + x w with the centered product (|x| <= 16q): acc stays an exact integer, below (1/2 + 2^-11) q
// times the number of terms (at most 4096 here) in magnitude.
__device__ __forceinline__ double mac_c(double acc, double x, double w, double q, double qinv) {
  return acc + mulmod_c_d(x, w, q, qinv);
}

// Inverse transform of the values x (positions 8g + k as above) through LDS, written to out in
// natural order; x signed accumulators (below 2^47 in magnitude; the signed inverse reduces them).
template <int GPT>
__device__ __forceinline__ void ntt_inv_store(double* lds, const NttTab& T, const double (&x)[GPT][8], double* out) {
  const int n = 1 << T.logn;
  __syncthreads();  // earlier readers of LDS are done
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int g = threadIdx.x + j * blockDim.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) lds[8 * g + k] = x[j][k];
  }
  __syncthreads();
  ntt_inv_lds_c(lds, T);
  for (int v = threadIdx.x; v < n; v += blockDim.x) out[v] = lds[v];
}

// Workgroup (col, z): the ring switch of ciphertext col in slot z, before RS_p:
// Aring = sum_{i, r} d_{i,r} K~mask_{z,i,r},  Bring = sum_{i, r} d_{i,r} K~key_{z,i,r}  (in R_{N_Q}).
template <int GPT, int S0>
__global__ void __launch_bounds__(kNttThreads)
k_fs_ring(FsConsts C, int64_t ncols, const double* Dg, const double* rk, double* Aring, double* Bring) {
  extern __shared__ double lds[];
  const int64_t G = ncols * C.nz;
  const int64_t f = xcd_item(blockIdx.x, G);
  if (f >= G) return;
  const int64_t col = f / C.nz;
  const int z = (int)(f - col * C.nz);
  const int nq = 1 << C.logn_q;
  const NttTab& T = C.tab[z];
  const double q = C.zd[z], qinv = C.zinv[z];
  double accA[GPT][8], accB[GPT][8], x[GPT][8];
#pragma unroll
  for (int j = 0; j < GPT; ++j)
#pragma unroll
    for (int k = 0; k < 8; ++k) accA[j][k] = accB[j][k] = 0.0;
  for (int i = 0; i <= C.level; ++i) {
    for (int r = 0; r < C.rho; ++r) {
      const double* src = Dg + (((size_t)col * (C.level + 1) + i) * C.rho + r) * nq;
      ntt_fwd_fused<GPT, S0>(lds, T, [&](int pos) { return src[pos]; }, x);  // digits below q_i < 2z
      const double* ka = rk + (((size_t)z * (C.level + 1) + i) * 2 * C.rho + r) * nq;
      const double* kb = ka + (size_t)C.rho * nq;
#pragma unroll
      for (int j = 0; j < GPT; ++j) {
        const int v0 = 8 * (threadIdx.x + j * blockDim.x);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          accA[j][k] = mac_c(accA[j][k], x[j][k], ka[v0 + k], q, qinv);
          accB[j][k] = mac_c(accB[j][k], x[j][k], kb[v0 + k], q, qinv);
        }
      }
    }
  }
  ntt_inv_store<GPT>(lds, T, accA, Aring + ((size_t)z * ncols + col) * nq);
  ntt_inv_store<GPT>(lds, T, accB, Bring + ((size_t)z * ncols + col) * nq);
}

// Workgroup (c, z, g): the conversion of column c's k chunks in slot z, before RS_p, for the outputs
// j' in [2g, 2g + 2) (and the shared mask when g = 0):
// Aconv = sum_{i, j} d_i(a'_j) k_ij,  Bconv_j' = sum_{i, j} d_i(a'_j) beta_ij'.
// The chunks' masks a'_j = RS_p(Aring) and their digits are formed as the transforms load them.
template <int GPT, int S0>
__global__ void __launch_bounds__(kNttThreads)
k_fs_conv(FsConsts C, int64_t d3, const double* Aring, const double* ck, double* Aconv, double* Bconv) {
  extern __shared__ double lds[];
  const int groups = (C.k + 1) / 2;
  const int64_t G = d3 * C.nz * groups;
  const int64_t f = xcd_item(blockIdx.x, G);
  if (f >= G) return;
  const int64_t c = f / ((int64_t)C.nz * groups);
  const int zg = (int)(f - c * C.nz * groups);
  const int z = zg / groups, g = zg - (zg / groups) * groups;
  const int nq = 1 << C.logn_q;
  const int64_t ncols = d3 * C.k;
  const int l = C.level;
  const NttTab& T = C.tab[z];
  const double q = C.zd[z], qinv = C.zinv[z], pd = C.zd[l + 1];
  const int j0 = 2 * g;
  const int nb = C.k - j0 < 2 ? C.k - j0 : 2;
  double accA[GPT][8], accB0[GPT][8], accB1[GPT][8], x[GPT][8];
#pragma unroll
  for (int jj = 0; jj < GPT; ++jj)
#pragma unroll
    for (int k = 0; k < 8; ++k) accA[jj][k] = accB0[jj][k] = accB1[jj][k] = 0.0;
  for (int j = 0; j < C.k; ++j) {
    const int64_t col = c * C.k + j;
    const double* Ap = Aring + ((size_t)(l + 1) * ncols + col) * nq;
    for (int i = 0; i <= l; ++i) {
      const double* Ai = Aring + ((size_t)i * ncols + col) * nq;
      const double qi = C.zd[i], qiinv = C.zinv[i], pinv = C.pinv[i], gh = C.ghat[i];
      ntt_fwd_fused<GPT, S0>(
          lds, T,
          [&](int v) { return mulmod_d(rs_d(Ai[v], Ap[v], pd, qi, qiinv, pinv), gh, qi, qiinv); }, x);
      const double* kk = ck + (((size_t)z * (l + 1) + i) * C.k + j) * (1 + C.k) * nq;
      const double* kb0 = kk + (size_t)(1 + j0) * nq;
      const double* kb1 = kk + (size_t)(nb > 1 ? 2 + j0 : 1 + j0) * nq;
#pragma unroll
      for (int jj = 0; jj < GPT; ++jj) {
        const int v0 = 8 * (threadIdx.x + jj * blockDim.x);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const double xv = x[jj][k];
          if (g == 0) accA[jj][k] = mac_c(accA[jj][k], xv, kk[v0 + k], q, qinv);
          accB0[jj][k] = mac_c(accB0[jj][k], xv, kb0[v0 + k], q, qinv);
          if (nb > 1) accB1[jj][k] = mac_c(accB1[jj][k], xv, kb1[v0 + k], q, qinv);
        }
      }
    }
  }
  if (g == 0) ntt_inv_store<GPT>(lds, T, accA, Aconv + ((size_t)z * d3 + c) * nq);
  ntt_inv_store<GPT>(lds, T, accB0, Bconv + (((size_t)z * d3 + c) * C.k + j0) * nq);
  if (nb > 1) ntt_inv_store<GPT>(lds, T, accB1, Bconv + (((size_t)z * d3 + c) * C.k + j0 + 1) * nq);
}

// Element (c, u): RS_p of the converted parts, the ring-switched b' = b(rho u) + RS_p(Bring), and
// RS_{q_l} down to q_0 .. q_{l-1}; written as the query ciphertext row c = [b_0 .. b_{k-1} (first d2) | a].
__global__ void k_fs_finish(FsConsts C, const uint64_t* T, int64_t d3, const double* Bring, const double* Aconv,
                            const double* Bconv, uint64_t* XT, int64_t K) {
  const int nq = 1 << C.logn_q;
  const int64_t nt = (int64_t)nq * C.rho;
  const int64_t ncols = d3 * C.k;
  const int l = C.level;
  const double pd = C.zd[l + 1], ql = C.zd[l];
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < d3 * nq; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = x / nq;
    const int u = (int)(x - c * nq);
    // the mask: a_i = RS_p(Aconv)_i for i <= l, then RS_{q_l}
    const double ap = Aconv[((size_t)(l + 1) * d3 + c) * nq + u];
    const double al = rs_d(Aconv[((size_t)l * d3 + c) * nq + u], ap, pd, ql, C.zinv[l], C.pinv[l]);
    for (int i = 0; i < l; ++i) {
      const double ai = rs_d(Aconv[((size_t)i * d3 + c) * nq + u], ap, pd, C.zd[i], C.zinv[i], C.pinv[i]);
      XT[((size_t)i * d3 + c) * K + C.d2 + u] = to_u(rs_d(ai, al, ql, C.zd[i], C.zinv[i], C.qlinv[i]));
    }
    // the bodies: chunk j' at code positions j' N_Q + u
    for (int jp = 0; jp < C.k; ++jp) {
      const int64_t t = (int64_t)jp * nq + u;
      if (t >= C.d2) break;
      const int64_t col = c * C.k + jp;
      const double brp = Bring[((size_t)(l + 1) * ncols + col) * nq + u];
      const double bcp = Bconv[(((size_t)(l + 1) * d3 + c) * C.k + jp) * nq + u];
      double bl = 0.0;
      for (int i = l; i >= 0; --i) {
        const double q = C.zd[i], qinv = C.zinv[i];
        const double bt = to_d(T[(((size_t)i * ncols + col) * 2 + 1) * nt + (int64_t)C.rho * u]);
        const double br = rs_d(Bring[((size_t)i * ncols + col) * nq + u], brp, pd, q, qinv, C.pinv[i]);
        const double bc = rs_d(Bconv[(((size_t)i * d3 + c) * C.k + jp) * nq + u], bcp, pd, q, qinv, C.pinv[i]);
        const double bi = addmod_d(addmod_d(bt, br, q), bc, q);
        if (i == l)
          bl = bi;
        else
          XT[((size_t)i * d3 + c) * K + t] = to_u(rs_d(bi, bl, ql, q, qinv, C.qlinv[i]));
      }
    }
  }
}

// The fused kernels: blockDim = N_Q / (8 GPT) threads (GPT = 2 at N_Q = 2^14, 1024 threads).
template <int GPT, int S0>
static hipError_t launch_fused_as(const FsConsts& C, int64_t ncols, int64_t d3, const FsWork& w, const double* rk,
                                  const double* ck, bool conv, hipStream_t s) {
  const size_t lds = sizeof(double) << C.logn_q;
  const int threads = (1 << C.logn_q) / (8 * GPT);
  if (!conv) {
    hipError_t e = allow_lds(k_fs_ring<GPT, S0>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fs_ring<GPT, S0>), dim3(xcd_grid(ncols * C.nz)), dim3(threads), lds, s, C, ncols, w.Dg,
                       rk, w.Aring, w.Bring);
  } else {
    hipError_t e = allow_lds(k_fs_conv<GPT, S0>, lds);
    if (e != hipSuccess) return e;
    const int groups = (C.k + 1) / 2;
    hipLaunchKernelGGL((k_fs_conv<GPT, S0>), dim3(xcd_grid(d3 * C.nz * groups)), dim3(threads), lds, s, C, d3,
                       w.Aring, ck, w.Aconv, w.Bconv);
  }
  return hipGetLastError();
}

static hipError_t launch_fused(const FsConsts& C, int64_t ncols, int64_t d3, const FsWork& w, const double* rk,
                               const double* ck, bool conv, hipStream_t s) {
  const int s0 = (C.logn_q - 1) % 3 + 1;
  if (C.logn_q <= 13) {
    if (s0 == 1) return launch_fused_as<1, 1>(C, ncols, d3, w, rk, ck, conv, s);
    if (s0 == 2) return launch_fused_as<1, 2>(C, ncols, d3, w, rk, ck, conv, s);
    return launch_fused_as<1, 3>(C, ncols, d3, w, rk, ck, conv, s);
  }
  return launch_fused_as<2, 2>(C, ncols, d3, w, rk, ck, conv, s);  // 2^14 = 2^(2 + 3 + 3 + 3 + 3)
}

hipError_t launch_fs_switch(const FsConsts& C, const uint64_t* T, int64_t d3, const double* rk, const double* ck,
                            const FsWork& w, uint64_t* XT, int64_t K, hipStream_t s, hipEvent_t* ev) {
  if (d3 <= 0) return hipSuccess;
  const int64_t ncols = d3 * C.k;
  const int nq = 1 << C.logn_q;
  if (ev) (void)hipEventRecord(ev[0], s);
  {
    hipLaunchKernelGGL(k_fs_digits, dim3((unsigned)(ncols * (C.level + 1))), dim3(256), 0, s, C, T, ncols, w.Dg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  hipError_t e = launch_fused(C, ncols, d3, w, rk, ck, false, s);
  if (e != hipSuccess) return e;
  if (ev) (void)hipEventRecord(ev[2], s);
  e = launch_fused(C, ncols, d3, w, rk, ck, true, s);
  if (e != hipSuccess) return e;
  if (ev) (void)hipEventRecord(ev[3], s);
  {
    const int64_t n = d3 * nq;
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_fs_finish, dim3((unsigned)blocks), dim3(256), 0, s, C, T, d3, w.Bring, w.Aconv, w.Bconv,
                       XT, K);
    e = hipGetLastError();
  }
  if (ev) (void)hipEventRecord(ev[4], s);
  return e;
}

}  // namespace hfe
