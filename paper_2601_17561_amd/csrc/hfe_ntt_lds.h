// LDS-resident negacyclic NTT (ring degrees up to 2^14) shared by the kernels that transform one
// polynomial per workgroup: the merged transforms of Longa and Naehrig (2016), forward Cooley-Tukey
// with twiddles psi^brv(i) (output in bit-reversed order), inverse Gentleman-Sande with psi^-brv(i)
// and a final 1/n scale.  Residues mod a 36-bit prime are held as doubles (exact integers below 2^36)
// and multiplied with the error-free fp64 product mulmod_d of hfe_exact.h.
#pragma once
#include <type_traits>

#include "hfe_internal.h"

namespace hfe {
constexpr int kNttThreads = 1024;

// ------------------------------------------------------------------ fp64 residue arithmetic
// Residues mod q < 2^36 as doubles holding exact integers in [0, q); products by mulmod_d
// (hfe_exact.h).
__device__ __forceinline__ double to_d(uint64_t x) { return (double)x; }    // exact below 2^53
__device__ __forceinline__ uint64_t to_u(double x) { return (uint64_t)x; }  // x an integer in [0, q)

// The transforms address the array through an accessor A: a plain double* (natural layout) or SwLds,
// the same N values with each aligned row of 32 permuted (index i at i ^ h(i >> 5)).  A round whose stride
// is below 32 has the 64 lanes of a wavefront read 2^S values each at addresses 2t or 8 apart, which in
// the natural layout fall into 4 to 8 of the LDS banks; h spreads the rows over the banks so that every
// round of a transform of degree 2^14 reads and writes whole bank rows (in both halves of a wavefront for
// 32 banks, and for 64), and no round of smaller degrees meets more than two-way conflicts.  Kernels that
// use SwLds address the array through it everywhere, so the permutation is invisible to them.
// h is linear over GF(2), so the place of i ^ j for indices with disjoint bits is the XOR of their places:
// a round computes the place of its group's base once and reaches the other 2^S - 1 values with one XOR
// by a constant of the round (lds_place of k stride).
struct SwLds {
  double* p;
  __device__ __forceinline__ static int h(int r) {
    return (r & 7) | ((((r >> 3) ^ r) & 1) << 3) | (((r >> 1) & 1) << 4);
  }
  __device__ __forceinline__ double& operator[](int i) const { return p[i ^ h(i >> 5)]; }
};

// The byte offset of logical index i in the array (its place times 8) and the value at a byte offset, for
// both accessors; XORs of places are XORs of their byte offsets.
__device__ __forceinline__ uint32_t lds_place(const double*, int i) { return (uint32_t)i << 3; }
__device__ __forceinline__ uint32_t lds_place(const SwLds&, int i) { return (uint32_t)(i ^ SwLds::h(i >> 5)) << 3; }
__device__ __forceinline__ double& lds_at(double* a, uint32_t b) {
  return *reinterpret_cast<double*>(reinterpret_cast<char*>(a) + b);
}
__device__ __forceinline__ double& lds_at(const SwLds& a, uint32_t b) {
  return *reinterpret_cast<double*>(reinterpret_cast<char*>(a.p) + b);
}

// Both transforms run in rounds of up to three butterfly stages: a thread loads a group of 2^S
// coefficients into registers, applies S stages there and stores them back, so a transform of
// degree 2^logn takes ceil(logn / 3) LDS passes and barriers instead of logn.
//
// Forward (Cooley-Tukey) round with first half-size t: group g holds a[base + k stride], k < 2^S,
// stride = t / 2^(S-1), base = B 2t + r (B = g / stride, r = g mod stride).  Stage s (half-size
// t / 2^s, m = n / (2t) 2^s blocks) pairs k and k + 2^(S-1-s); the pair lies in block
// B 2^s + (k >> (S - s)), whose twiddle is psi[m + block].
// The S stages of one forward round on the group held in registers x[0 .. 2^S) (first twiddle block
// m1 = n / (2t), group block B as above).
template <int S>
__device__ __forceinline__ void fwd_stages(double* x, const NttTab& T, int m1, int B) {
  constexpr int G = 1 << S;
  const double q = T.qd, qinv = T.qinv;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int h = 1 << (S - 1 - s);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (k & h) continue;
      const uint32_t w = (uint32_t)((m1 << s) + (B << s) + (k >> (S - s)));
      const double U = x[k];
      const double V = mulmod_d(x[k + h], T.psi_d[w], q, qinv);
      x[k] = addmod_d(U, V, q);
      x[k + h] = submod_d(U, V, q);
    }
  }
}

// The same stages on signed values (ct_butterfly_c): each stage adds at most about q/2 to the magnitude.
template <int S>
__device__ __forceinline__ void fwd_stages_c(double* x, const NttTab& T, int m1, int B) {
  constexpr int G = 1 << S;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int h = 1 << (S - 1 - s);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (k & h) continue;
      const uint32_t w = (uint32_t)((m1 << s) + (B << s) + (k >> (S - s)));
      ct_butterfly_c(x[k], x[k + h], T.psi_d[w], T.qd, T.qinv);
    }
  }
}

template <int S, class A>
__device__ __forceinline__ void fwd_round_c(A a, const NttTab& T, int n, int t) {
  constexpr int G = 1 << S;
  const int ls = __builtin_ctz((unsigned)t) - (S - 1);  // stride = 2^ls (t, n powers of two)
  const int stride = 1 << ls, m1 = n / (2 * t);
  uint32_t off[G];  // byte offsets of k stride (bits disjoint from any base)
#pragma unroll
  for (int k = 0; k < G; ++k) off[k] = lds_place(a, k << ls);
  for (int g = threadIdx.x; g < (n >> S); g += blockDim.x) {
    const int B = g >> ls, r = g & (stride - 1);
    const uint32_t p0 = lds_place(a, (B << (ls + S)) + r);  // base = B 2t + r
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = lds_at(a, p0 ^ off[k]);
    fwd_stages_c<S>(x, T, m1, B);
#pragma unroll
    for (int k = 0; k < G; ++k) lds_at(a, p0 ^ off[k]) = x[k];
  }
  __syncthreads();
}

template <int S, class A>
__device__ __forceinline__ void fwd_round(A a, const NttTab& T, int n, int t) {
  constexpr int G = 1 << S;
  const int ls = __builtin_ctz((unsigned)t) - (S - 1);  // stride = 2^ls (t, n powers of two)
  const int stride = 1 << ls, m1 = n / (2 * t);
  uint32_t off[G];  // byte offsets of k stride (bits disjoint from any base)
#pragma unroll
  for (int k = 0; k < G; ++k) off[k] = lds_place(a, k << ls);
  for (int g = threadIdx.x; g < (n >> S); g += blockDim.x) {
    const int B = g >> ls, r = g & (stride - 1);
    const uint32_t p0 = lds_place(a, (B << (ls + S)) + r);  // base = B 2t + r
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = lds_at(a, p0 ^ off[k]);
    fwd_stages<S>(x, T, m1, B);
#pragma unroll
    for (int k = 0; k < G; ++k) lds_at(a, p0 ^ off[k]) = x[k];
  }
  __syncthreads();
}

// Inverse (Gentleman-Sande) round with first half-size t: group g holds a[base + k t], k < 2^S,
// base = B 2^S t + r (B = g / t, r = g mod t).  Stage s (half-size 2^s t, m = n / (2^(s+1) t)
// blocks) pairs k and k + 2^s; the pair lies in block B 2^(S-1-s) + (k >> (s + 1)), twiddle
// ipsi[m + block].  With scale, the round ends with the 1/n factor.
template <int S, class A>
__device__ __forceinline__ void inv_round(A a, const NttTab& T, int n, int t, bool scale) {
  constexpr int G = 1 << S;
  const double q = T.qd, qinv = T.qinv;
  const int lt = __builtin_ctz((unsigned)t);
  uint32_t off[G];  // byte offsets of k t (bits disjoint from any base)
#pragma unroll
  for (int k = 0; k < G; ++k) off[k] = lds_place(a, k << lt);
  for (int g = threadIdx.x; g < (n >> S); g += blockDim.x) {
    const int B = g >> lt, r = g & (t - 1);
    const uint32_t p0 = lds_place(a, (B << (lt + S)) + r);  // base = B 2^S t + r
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = lds_at(a, p0 ^ off[k]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int h = 1 << s;
      const int m = n / (2 * h * t);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (k & h) continue;
        const uint32_t w = (uint32_t)(m + (B << (S - 1 - s)) + (k >> (s + 1)));
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
    for (int k = 0; k < G; ++k) lds_at(a, p0 ^ off[k]) = x[k];
  }
  __syncthreads();
}

// The inverse round on signed values: the round first takes its values (any integers below 2^47 in
// magnitude) to centered representatives (reduce_c_d, at most (1/2 + 2^-11) q), so that its S <= 3
// Gentleman-Sande stages (X + Y, and (X - Y) W centered) keep every value below 4.01q and every
// product operand below 8.02q; the last round scales by 1/n and returns residues in [0, q).
template <int S, class A>
__device__ __forceinline__ void inv_round_c(A a, const NttTab& T, int n, int t, bool last) {
  constexpr int G = 1 << S;
  const double q = T.qd, qinv = T.qinv;
  const int lt = __builtin_ctz((unsigned)t);
  uint32_t off[G];  // byte offsets of k t (bits disjoint from any base)
#pragma unroll
  for (int k = 0; k < G; ++k) off[k] = lds_place(a, k << lt);
  for (int g = threadIdx.x; g < (n >> S); g += blockDim.x) {
    const int B = g >> lt, r = g & (t - 1);
    const uint32_t p0 = lds_place(a, (B << (lt + S)) + r);  // base = B 2^S t + r
    double x[G];
#pragma unroll
    for (int k = 0; k < G; ++k) x[k] = reduce_c_d(lds_at(a, p0 ^ off[k]), q, qinv);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int h = 1 << s;
      const int m = n / (2 * h * t);
#pragma unroll
      for (int k = 0; k < G; ++k) {
        if (k & h) continue;
        const uint32_t w = (uint32_t)(m + (B << (S - 1 - s)) + (k >> (s + 1)));
        const double U = x[k], V = x[k + h];
        x[k] = U + V;
        x[k + h] = mulmod_c_d(U - V, T.ipsi_d[w], q, qinv);
      }
    }
    if (last) {
#pragma unroll
      for (int k = 0; k < G; ++k) x[k] = residue_of_c(mulmod_c_d(x[k], T.n_inv_d, q, qinv), q);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) lds_at(a, p0 ^ off[k]) = x[k];
  }
  __syncthreads();
}

// Forward negacyclic NTT in place (output in bit-reversed order).
template <class A>
__device__ __forceinline__ void ntt_fwd_lds(A a, const NttTab& T) {
  const int n = 1 << T.logn;
  int t = n >> 1, left = T.logn;
  while (left > 0) {
    if (left >= 3) {
      fwd_round<3>(a, T, n, t);
      t >>= 3;
      left -= 3;
    } else if (left == 2) {
      fwd_round<2>(a, T, n, t);
      t >>= 2;
      left -= 2;
    } else {
      fwd_round<1>(a, T, n, t);
      t >>= 1;
      left -= 1;
    }
  }
}

// The same transform on signed values without corrections (fwd_round_c): inputs in [0, q) give
// outputs congruent to the exact ones, below 8.1q in magnitude for degrees up to 2^14.
template <class A>
__device__ __forceinline__ void ntt_fwd_lds_c(A a, const NttTab& T) {
  const int n = 1 << T.logn;
  int t = n >> 1, left = T.logn;
  while (left > 0) {
    if (left >= 3) {
      fwd_round_c<3>(a, T, n, t);
      t >>= 3;
      left -= 3;
    } else if (left == 2) {
      fwd_round_c<2>(a, T, n, t);
      t >>= 2;
      left -= 2;
    } else {
      fwd_round_c<1>(a, T, n, t);
      t >>= 1;
      left -= 1;
    }
  }
}

// The inverse on signed inputs (any integers below 2^47 in magnitude) through inv_round_c; outputs in
// [0, q), the same residues as ntt_inv_lds of the inputs' residues.
template <class A>
__device__ __forceinline__ void ntt_inv_lds_c(A a, const NttTab& T) {
  const int n = 1 << T.logn;
  int t = 1, left = T.logn;
  while (left > 0) {
    if (left >= 3) {
      inv_round_c<3>(a, T, n, t, left == 3);
      t <<= 3;
      left -= 3;
    } else if (left == 2) {
      inv_round_c<2>(a, T, n, t, true);
      t <<= 2;
      left -= 2;
    } else {
      inv_round_c<1>(a, T, n, t, true);
      t <<= 1;
      left -= 1;
    }
  }
}

// Inverse negacyclic NTT in place (input in bit-reversed order), including the 1/n factor.
template <class A>
__device__ __forceinline__ void ntt_inv_lds(A a, const NttTab& T) {
  const int n = 1 << T.logn;
  int t = 1, left = T.logn;
  while (left > 0) {
    if (left >= 3) {
      inv_round<3>(a, T, n, t, left == 3);
      t <<= 3;
      left -= 3;
    } else if (left == 2) {
      inv_round<2>(a, T, n, t, true);
      t <<= 2;
      left -= 2;
    } else {
      inv_round<1>(a, T, n, t, true);
      t <<= 1;
      left -= 1;
    }
  }
}

// Forward transforms fused with their load and their use.  With blockDim = n / (8 GPT), the first
// round (S0 = (log n - 1) mod 3 + 1 stages, t = n / 2: group g holds the coefficients g + k n / 2^S0)
// reads its coefficients from global memory into registers, the middle rounds of three stages run
// through LDS, and the last round (t = 4: group g holds the contiguous coefficients 8g .. 8g + 7 of
// the bit-reversed output) stays in registers, where the caller multiplies by the keys: two LDS
// passes and two barriers fewer per transform than a load, the transform and a reload.  The
// butterflies run on signed values without corrections (ct_butterfly_c, hfe_exact.h): inputs below 2q
// leave a transform of degree up to 2^14 below 9.1q, congruent to the
// exact outputs, which the centered products of the multiply-accumulate take as they are.
// First round: loads every value this thread's groups need (before the barrier that lets it
// overwrite LDS), then the S0 stages and the store.
template <int GPT, int S0, class Load>
__device__ __forceinline__ void fused_first_round(double* lds, const NttTab& T, Load load) {
  constexpr int G = 1 << S0;
  constexpr int M = 8 * GPT / G;  // groups per thread
  const int n = 1 << T.logn, ng = n >> S0;
  double y[M][G];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int k = 0; k < G; ++k) y[m][k] = load(threadIdx.x + m * blockDim.x + k * ng);
  __syncthreads();  // the previous transform's last round has read LDS
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int g = threadIdx.x + m * blockDim.x;
    fwd_stages_c<S0>(y[m], T, 1, 0);
#pragma unroll
    for (int k = 0; k < G; ++k) lds[g + k * ng] = y[m][k];
  }
  __syncthreads();
}

template <int GPT, int S0, class Load>
__device__ __forceinline__ void ntt_fwd_fused(double* lds, const NttTab& T, Load load, double (&x)[GPT][8]) {
  const int n = 1 << T.logn;
  fused_first_round<GPT, S0>(lds, T, load);
  for (int t = (n >> 1) >> S0; t > 4; t >>= 3) fwd_round_c<3>(lds, T, n, t);
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int g = threadIdx.x + j * blockDim.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) x[j][k] = lds[8 * g + k];
    fwd_stages_c<3>(x[j], T, n >> 3, g);
  }
}

// A pass over the n values of a workgroup's polynomial (thread t takes t, t + blockDim, ...; staged_range:
// the indices lo .. hi - 1 the same way) in chunks of CH per thread: the chunk's global loads (ld(i) returns
// what index i needs) are all issued before the first is used (st(i, loaded)), so that a thread waits for
// memory once per chunk rather than once per value.  With one workgroup per CU (a polynomial of 2^14 doubles
// fills the LDS) no other workgroup hides those waits.
template <int CH, class Ld, class St>
__device__ __forceinline__ void staged_range(int64_t lo, int64_t hi, Ld ld, St st) {
  using V = decltype(ld(lo));
  for (int64_t t0 = lo + threadIdx.x; t0 < hi; t0 += CH * (int64_t)blockDim.x) {
    V v[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int64_t t = t0 + j * (int64_t)blockDim.x;
      if (t < hi) v[j] = ld(t);
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int64_t t = t0 + j * (int64_t)blockDim.x;
      if (t < hi) st(t, v[j]);
    }
  }
}
template <int CH, class Ld, class St>
__device__ __forceinline__ void staged_pass(int n, Ld ld, St st) {
  using V = decltype(ld(0));
  for (int t0 = threadIdx.x; t0 < n; t0 += CH * blockDim.x) {
    V v[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int t = t0 + j * blockDim.x;
      if (t < n) v[j] = ld(t);
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int t = t0 + j * blockDim.x;
      if (t < n) st(t, v[j]);
    }
  }
}

static int ntt_block(int logn) {
  int half = 1 << (logn > 0 ? logn - 1 : 0);
  int b = half < 64 ? 64 : half;
  return b > kNttThreads ? kNttThreads : b;
}

template <class K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// R: NTT-domain coefficients each thread keeps in registers, n / blockDim (1 .. 16 for n <= 2^14),
// a template parameter so that the register arrays are no larger than the transform needs.
static int regs_per_thread(int logn) {
  const int r = (1 << logn) / ntt_block(logn);
  return r < 1 ? 1 : r;
}
// f(std::integral_constant<int, R>{}) for the runtime count r
template <class F>
static hipError_t by_regs(int r, F f) {
  switch (r) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hfe
