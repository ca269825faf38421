// Normalise and fold (Algorithm 2, Section 4.3, Appendix C.2): the kernels of a small CKKS evaluator at
// ring degree N <= 2^14 over the slots q_0 .. q_4 and the special prime p (slot 5).
//
// Ciphertexts are kept in the NTT domain as uint64 residues, [item][part (b, a)][slot][N]; every
// transform is one polynomial per workgroup in LDS (hfe_ntt_lds.h).  The operations a fold needs are
// built from a few passes:
//   k_fold_encode     the slot encoder (plaintext coefficients from integer slot values, hfe_slots.h)
//   k_fold_fwd        signed coefficients -> NTT-domain residues, for several slots
//   k_fold_inv        NTT-domain residues (or the product of two, or with a plaintext)
//                     -> coefficients (residues, centered, or the digits of a key switch)
//   k_fold_ks_mac     sum_i NTT(d_i) K_i for one slot: each digit's transform in LDS, the products
//                     accumulated in registers; the special prime's sum is transformed back and centered
//   k_fold_lift       (x k - NTT([y]_div)) div^-1 plus addends on every kept slot: RS_div of a product, of a
//                     constant times a ciphertext (with a mod-drop and an added constant), and the end of a
//                     key switch (with the tensor terms d0, d1 of a product, or sigma(b) of a rotation), and of
//                     a plaintext product (the normalisation, the product formed on load)
//   elementwise       the automorphism of a rotation as a permutation of the NTT points,
//                     group sums, key and input draws
#include "hfe_ntt_lds.h"
#include "hfe_slots.h"

namespace hfe {
namespace {

__device__ __forceinline__ double mm_d(double a, double b, int z, const FoldConsts& C) {
  return mulmod_d(a, b, C.zd[z], C.zinv[z]);
}

// ------------------------------------------------------------------ encoder
// Slot weights: w = v (mode 0, |v| <= 2^24) or round(2^30 / v) = floor((2^31 + v) / (2v)) (mode 1,
// 1 <= v <= 2^24); a value outside its range sets *bad and is replaced by 0 (mode 0) or 1 (mode 1).
__global__ void k_fold_weights(const int32_t* values, int64_t total, int mode, int64_t* w, uint32_t* bad) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = values[e];
    if (mode) {
      if (v < 1 || v > (1 << 24)) {
        atomicOr(bad, 1u);
        v = 1;
      }
      w[e] = ((int64_t(1) << 31) + v) / (2 * v);
    } else {
      if (v < -(1 << 24) || v > (1 << 24)) {
        atomicOr(bad, 1u);
        v = 0;
      }
      w[e] = v;
    }
  }
}

// The slot encoder (hfe_slots.h), one workgroup per item c: the M = N/2 slot values w[c][j] 2^e enter an
// inverse DFT of length M at bit-reversed positions pos[j] in LDS (real and imaginary parts, N doubles),
// log2 M radix-2 stages, then the untwist and the rounding: out[c][i], out[c][M + i].
__global__ void __launch_bounds__(kNttThreads) k_fold_encode(const int64_t* w, int logn, double scale,
                                                           const double* W, const double* Z, const int32_t* pos,
                                                           int64_t* out) {
  extern __shared__ double lds[];
  const int M = 1 << (logn - 1);
  double* xr = lds;
  double* xi = lds + M;
  const int64_t c = blockIdx.x;
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const int p = pos[j];
    xr[p] = (double)w[c * M + j] * scale;  // exact: |w| < 2^31, scale a power of two
    xi[p] = 0.0;
  }
  __syncthreads();
  for (int half = 1, lh = 0; half < M; half *= 2, ++lh) {
    const int step = M / (2 * half);
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int t = b & (half - 1);
      const int ia = ((b >> lh) << (lh + 1)) + t, ic = ia + half;
      slot_butterfly(xr[ia], xi[ia], xr[ic], xi[ic], W[2 * t * step], W[2 * t * step + 1]);
    }
    __syncthreads();
  }
  const double inv_m = 1.0 / (double)M;
  int64_t* o = out + c * 2 * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    double ur, ui;
    slot_untwist(xr[i], xi[i], Z[2 * i], Z[2 * i + 1], inv_m, ur, ui);
    o[i] = round_half_up(ur);
    o[M + i] = round_half_up(ui);
  }
}

// ------------------------------------------------------------------ transforms
// job = item * nsl + s: src[item * si + s * ss + t] (signed, |x| < 2^63) mod z_s -> forward NTT ->
// dst[item * di + s * ds + t].
__global__ void __launch_bounds__(kNttThreads) k_fold_fwd(FoldConsts C, const int64_t* src, int64_t si, int64_t ss,
                                                        uint64_t* dst, int64_t di, int64_t ds, SlotMap zm, int nsl) {
  extern __shared__ double lds_raw[];
  const SwLds lds{lds_raw};
  const int n = 1 << C.logn;
  const int64_t item = blockIdx.x / nsl;
  const int s = blockIdx.x - (int)(item * nsl);
  const int z = zm.z[s];
  const Mod md = C.mod[z];
  const int64_t* x = src + item * si + s * ss;
  staged_pass<4>(n, [&](int t) { return x[t]; }, [&](int t, int64_t v) { lds[t] = to_d(from_signed(v, md.q, md.mu)); });
  __syncthreads();
  ntt_fwd_lds_c(lds, C.tab[z]);
  uint64_t* y = dst + item * di + s * ds;
  const double zd = C.zd[z], zi = C.zinv[z];
  for (int t = threadIdx.x; t < n; t += blockDim.x) y[t] = to_u(residue_of_c(reduce_c_d(lds[t], zd, zi), zd));
}

// job = item * nsl + s: inverse NTT of src[item * si + s * ss] mod z_s (times the plaintext pm at slot z_s
// when pm is given, times y at the same place when y is given); mode 0: residues (uint64), 1: centered (int64),
// 2: residues times factor[s] mod z_s (the digits of a key switch).
__global__ void __launch_bounds__(kNttThreads) k_fold_inv(FoldConsts C, FoldInv a) {
  extern __shared__ double lds_raw[];
  const SwLds lds{lds_raw};
  const int n = 1 << C.logn;
  const int64_t item = blockIdx.x / a.nsl;
  const int s = blockIdx.x - (int)(item * a.nsl);
  const int z = a.zm.z[s];
  const int64_t off = item * a.si + s * a.ss;
  const uint64_t* x = a.src + off;
  if (a.pm) {  // the plaintext product formed on load
    const uint64_t* y = a.pm + (item >> 1) * a.pmi + (int64_t)z * n;
    struct Two {
      uint64_t x, y;
    };
    staged_pass<4>(n, [&](int t) { return Two{x[t], y[t]}; },
                   [&](int t, const Two& v) { lds[t] = mm_d(to_d(v.x), to_d(v.y), z, C); });
  } else if (a.y) {
    const uint64_t* y = a.y + off;
    struct Two {
      uint64_t x, y;
    };
    staged_pass<4>(n, [&](int t) { return Two{x[t], y[t]}; },
                   [&](int t, const Two& v) { lds[t] = mm_d(to_d(v.x), to_d(v.y), z, C); });
  } else {
    staged_pass<4>(n, [&](int t) { return x[t]; }, [&](int t, uint64_t v) { lds[t] = to_d(v); });
  }
  __syncthreads();
  ntt_inv_lds_c(lds, C.tab[z]);
  const int64_t doff = item * a.di + s * a.ds;
  if (a.mode == 1) {
    int64_t* y = static_cast<int64_t*>(a.dst) + doff;
    for (int t = threadIdx.x; t < n; t += blockDim.x) y[t] = centered(to_u(lds[t]), C.mod[z].q);
  } else {
    uint64_t* y = static_cast<uint64_t*>(a.dst) + doff;
    const double fz = a.f.v[s];
    for (int t = threadIdx.x; t < n; t += blockDim.x) y[t] = to_u(a.mode == 2 ? mm_d(lds[t], fz, z, C) : lds[t]);
  }
}

// ------------------------------------------------------------------ key switching
// job = s * items + item (slot-major: the blocks that run together share the slot's keys, (level + 1) pairs of
// N doubles, which stay in each XCD's L2), slot z = s (s <= level) or p (s = level + 1).  For each digit i <= level
// (dig[item][i][N], residues mod q_i): reduce mod z, forward NTT in LDS, multiply by the key's two
// parts for (z, i) and accumulate in registers (R coefficients per thread and part).  At z = q_i the
// digit's transform is the NTT-domain value it came from times its factor (src [times y] at slot i, times
// dg.f[i], as the digit pass k_fold_inv with mode 2 describes it), taken directly.  The key of the
// item is keys + kidx[item] * kstride (kidx NULL: key 0), laid out [s][i][2][N] doubles.  Slots of Q_l
// store the NTT-domain sums to acc[item][part][s][N]; the special prime's sums are transformed back,
// centered and stored to accp[item][part][N].
template <int R>
__global__ void __launch_bounds__(kNttThreads) k_fold_ks_mac(FoldConsts C, int level, FoldInv dg,
                                                           const uint64_t* dig, const double* keys, int64_t kstride,
                                                           const int32_t* kidx, uint64_t* acc, int64_t* accp) {
  extern __shared__ double lds_raw[];
  const SwLds lds{lds_raw};
  const int n = 1 << C.logn;
  const int nsl = level + 2;
  const int64_t items = gridDim.x / nsl;
  const int s = (int)(blockIdx.x / items);
  const int64_t item = blockIdx.x - s * items;
  const bool special = s == level + 1;
  const int z = special ? 5 : s;
  const Mod md = C.mod[z];
  const double* key = keys + (kidx ? (int64_t)kidx[item] : 0) * kstride + (int64_t)s * (level + 1) * 2 * n;
  // signed transforms: each digit's transform is below 8.1z in magnitude, each product centered within
  // (1/2 + 2^-11) z, so the sums over at most 4 digits stay below 2.1z
  const double zd = C.zd[z], zi = C.zinv[z];
  double ab[R], aa[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ab[r] = aa[r] = 0.0;
  for (int i = 0; i <= level; ++i) {
    if (i == s) {  // the digit's own prime: its transform is the NTT-domain value it came from
      const int64_t off = item * dg.si + i * dg.ss;
      const uint64_t* x = dg.src + off;
      const uint64_t* y = dg.y ? dg.y + off : nullptr;
      const double f = dg.f.v[i];
      struct Two {
        uint64_t x, y;
      };
      staged_pass<4>(n, [&](int t) { return Two{x[t], y ? y[t] : 0}; }, [&](int t, const Two& u) {
        double v = to_d(u.x);
        if (y) v = mm_d(v, to_d(u.y), z, C);
        lds[t] = mm_d(v, f, z, C);
      });
      __syncthreads();
    } else {
      const uint64_t* d = dig + (item * (level + 1) + i) * n;
      staged_pass<4>(n, [&](int t) { return d[t]; }, [&](int t, uint64_t v) { lds[t] = to_d(barrett64(v, md.q, md.mu)); });
      __syncthreads();
      ntt_fwd_lds_c(lds, C.tab[z]);
    }
    const double* kb = key + (int64_t)i * 2 * n;   // part 0: mask k_i, part 1: beta_i
    // four coefficients at a time: the scheduler may not hoist more key loads, which with the 2R live
    // sums would spill registers
#pragma unroll
    for (int r0 = 0; r0 < R; r0 += 4) {
#pragma unroll
      for (int r = r0; r < r0 + 4 && r < R; ++r) {
        const int t = threadIdx.x + r * blockDim.x;
        const double v = lds[t];
        aa[r] += mulmod_c_d(v, kb[t], zd, zi);
        ab[r] += mulmod_c_d(v, kb[n + t], zd, zi);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
  if (!special) {
    uint64_t* ob = acc + ((item * 2 + 0) * (level + 1) + s) * n;
    uint64_t* oa = acc + ((item * 2 + 1) * (level + 1) + s) * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = threadIdx.x + r * blockDim.x;
      ob[t] = to_u(residue_of_c(reduce_c_d(ab[r], zd, zi), zd));
      oa[t] = to_u(residue_of_c(reduce_c_d(aa[r], zd, zi), zd));
    }
    return;
  }
  for (int part = 0; part < 2; ++part) {
#pragma unroll
    for (int r = 0; r < R; ++r) lds[threadIdx.x + r * blockDim.x] = part ? aa[r] : ab[r];
    __syncthreads();
    ntt_inv_lds_c(lds, C.tab[z]);
    int64_t* o = accp + (item * 2 + part) * n;
    for (int t = threadIdx.x; t < n; t += blockDim.x) o[t] = centered(to_u(lds[t]), md.q);
    __syncthreads();
  }
}

// job = (item * 2 + part) * nsl + s, slot z = zm.z[s]:
// out = (x pm xmul[s] - NTT_z(cen mod z)) inv[s] + addends mod z (pm the plaintext at slot z when given), with
// cen = cen[(item * 2 + part) * N + t], or
// cen = the centered k u mod q_cl from the residues u = ures[(item * 2 + part) * N + t] when ures is given.
// Addends: add (part 0 only when ap = 0), add2 (both parts), the tensor terms of tx and ty (part 0: b_x b_y,
// part 1: a_x b_y + a_y b_x) and the constant cres on part 0.
__global__ void __launch_bounds__(kNttThreads) k_fold_lift(FoldConsts C, FoldLift a) {
  extern __shared__ double lds_raw[];
  const SwLds lds{lds_raw};
  const int n = 1 << C.logn;
  const int64_t ip = blockIdx.x / a.nsl;
  const int s = blockIdx.x - (int)(ip * a.nsl);
  const int64_t item = ip >> 1;
  const int part = (int)(ip & 1);
  const int z = a.zm.z[s];
  const Mod md = C.mod[z];
  if (a.ures) {  // the centered value of k u mod q_cl from the residues u (a constant's rescale)
    const uint64_t* u = a.ures + ip * n;
    const int cl = a.cl;
    const uint64_t qc = C.mod[cl].q;
    staged_pass<4>(n, [&](int t) { return u[t]; }, [&](int t, uint64_t v) {
      const int64_t cv = centered(to_u(mm_d(to_d(v), a.ku, cl, C)), qc);
      lds[t] = to_d(from_signed(cv, md.q, md.mu));
    });
  } else {
    const int64_t* c = a.cen + ip * n;
    staged_pass<4>(n, [&](int t) { return c[t]; },
                   [&](int t, int64_t v) { lds[t] = to_d(from_signed(v, md.q, md.mu)); });
  }
  __syncthreads();
  ntt_fwd_lds_c(lds, C.tab[z]);  // signed, below 8.1z
  const int64_t so = (int64_t)s * n;
  const uint64_t* xx = a.x + item * a.xi + part * a.xp + so;
  const uint64_t* aa = (a.add && (part == 0 || a.ap != 0)) ? a.add + item * a.ai + part * a.ap + so : nullptr;
  const uint64_t* a2 = a.add2 ? a.add2 + item * a.a2i + part * a.a2p + so : nullptr;
  const uint64_t* tx = a.tx ? a.tx + item * a.ti + so : nullptr;
  const uint64_t* ty = a.tx ? a.ty + item * a.ti + so : nullptr;
  uint64_t* o = a.out + item * a.oi + part * a.op + so;
  const double zd = C.zd[z], zi = C.zinv[z], w = a.inv.v[s];
  const double km = a.has_xmul ? a.xmul.v[s] : 0.0, kc = part == 0 ? a.cres.v[s] : 0.0;
  const uint64_t* pm = a.pm ? a.pm + item * a.pmi + (int64_t)z * n : nullptr;
  struct In {
    uint64_t x, pmv, ad, ad2, bx, by, ax, ay;
  };
  staged_pass<4>(
      n,
      [&](int t) {
        In r{xx[t], 0, 0, 0, 0, 0, 0, 0};
        if (pm) r.pmv = pm[t];
        if (aa) r.ad = aa[t];
        if (a2) r.ad2 = a2[t];
        if (tx) {
          r.bx = tx[t];
          r.by = ty[t];
          if (part != 0) {
            r.ax = tx[a.tp + t];
            r.ay = ty[a.tp + t];
          }
        }
        return r;
      },
      [&](int t, const In& r) {
        double xv = to_d(r.x);
        if (pm) xv = mm_d(xv, to_d(r.pmv), z, C);
        if (a.has_xmul) xv = mm_d(xv, km, z, C);
        double v = mulmod_c_d(xv - lds[t], w, zd, zi);  // |x - NTT| < 9.1z: centered product, below 0.51z
        v = v < 0.0 ? v + zd : v;                        // [0, z)
        if (aa) v = addmod_d(v, to_d(r.ad), zd);
        if (a2) v = addmod_d(v, to_d(r.ad2), zd);
        if (tx) {
          const double bx = to_d(r.bx), by = to_d(r.by);
          double d;
          if (part == 0) {
            d = mm_d(bx, by, z, C);
          } else {
            d = addmod_d(mm_d(to_d(r.ax), by, z, C), mm_d(to_d(r.ay), bx, z, C), zd);
          }
          if (a.has_tscale) d = mm_d(d, a.tscale.v[s], z, C);
          v = addmod_d(v, d, zd);
        }
        v = addmod_d(v, kc, zd);
        o[t] = to_u(v);
      });
}

// The end of a relinearised product divided by p q_l in one rounding: job = item * 2 + part,
// X = acc[item][part][l] + (p mod q_l) d (d the tensor's d0 or d1 at slot l, formed from tx, ty), its
// inverse transform r (mod q_l), and the value c = a + p ((r - a) p^-1 mod q_l) (a = accp, centered mod p),
// the representative of X modulo D = p q_l, centered: cen[item][part][t].
__global__ void __launch_bounds__(kNttThreads) k_fold_relin_center(FoldConsts C, int level, const uint64_t* acc,
                                                                 const int64_t* accp, const uint64_t* tx,
                                                                 const uint64_t* ty, double p_l, double pinv_l,
                                                                 int64_t D, int64_t* cen) {
  extern __shared__ double lds_raw[];
  const SwLds lds{lds_raw};
  const int n = 1 << C.logn;
  const int64_t ip = blockIdx.x;
  const int64_t item = ip >> 1;
  const int part = (int)(ip & 1);
  const int l = level;
  const int64_t per = (int64_t)(l + 1) * n;
  const uint64_t* x = acc + ip * per + (int64_t)l * n;
  const uint64_t* bx = tx + item * 2 * per + (int64_t)l * n;
  const uint64_t* by = ty + item * 2 * per + (int64_t)l * n;
  const double zd = C.zd[l];
  struct In {
    uint64_t x, bx, by, ax, ay;
  };
  staged_pass<4>(
      n,
      [&](int t) {
        In r{x[t], bx[t], by[t], 0, 0};
        if (part != 0) {
          r.ax = bx[per + t];
          r.ay = by[per + t];
        }
        return r;
      },
      [&](int t, const In& r) {
        double d;
        if (part == 0) {
          d = mm_d(to_d(r.bx), to_d(r.by), l, C);
        } else {
          d = addmod_d(mm_d(to_d(r.ax), to_d(r.by), l, C), mm_d(to_d(r.ay), to_d(r.bx), l, C), zd);
        }
        lds[t] = addmod_d(to_d(r.x), mm_d(d, p_l, l, C), zd);
      });
  __syncthreads();
  ntt_inv_lds_c(lds, C.tab[l]);
  const Mod ml = C.mod[l];
  const int64_t p = (int64_t)C.mod[5].q;
  const int64_t* ap = accp + ip * n;
  int64_t* o = cen + ip * n;
  staged_pass<4>(n, [&](int t) { return ap[t]; }, [&](int t, int64_t a) {
    const double am = to_d(from_signed(a, ml.q, ml.mu));
    const double u = mm_d(submod_d(lds[t], am, zd), pinv_l, l, C);  // (r - a) p^-1 mod q_l
    int64_t v = a + p * (int64_t)u;                                  // in (-p/2, D): |v| < 2^60
    if (v > D / 2) v -= D;
    o[t] = v;
  });
}

// ------------------------------------------------------------------ elementwise
// Rotation's automorphism on gathered items with nsl slots: out[u][part][s][t] =
// x[src[u]][part][s][perm[amt[u]][t]] (the NTT points of every prime are ordered alike).
__global__ void k_fold_perm(FoldConsts C, const uint64_t* x, const int32_t* src, const int32_t* amt,
                            const int32_t* perm, uint64_t* out, int64_t items, int nsl) {
  const int n = 1 << C.logn;
  const int64_t per = 2 * (int64_t)nsl * n;
  const int64_t total = items * per;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(e & (n - 1));
    const int64_t u = e / per, w = e - u * per;
    out[e] = x[(int64_t)src[u] * per + (w - t) + perm[(int64_t)amt[u] * n + t]];
  }
}

// Group sums of items with nsl slots: out[g] = sum over the members of group g; members are listed in
// mem[beg[g] .. beg[g+1]) as idx * 2 + (rotated ? 1 : 0), rotated[idx] or f[idx].
__global__ void k_fold_group_sum(FoldConsts C, const uint64_t* f, const uint64_t* rotated, const int32_t* beg,
                                 const int32_t* mem, uint64_t* out, int64_t groups, int nsl) {
  const int n = 1 << C.logn;
  const int64_t per = 2 * (int64_t)nsl * n;
  const int64_t total = groups * per;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = e / per, w = e - g * per;
    const double zd = C.zd[(int)((w >> C.logn) % nsl)];
    double v = 0.0;
    for (int m = beg[g]; m < beg[g + 1]; ++m) {
      const int32_t code = mem[m];
      const uint64_t* b = (code & 1) ? rotated : f;
      v = addmod_d(v, to_d(b[(int64_t)(code >> 1) * per + w]), zd);
    }
    out[e] = to_u(v);
  }
}

// Scatter rotated items back: x[dst[u]] = y[u] (items with nsl slots).
__global__ void k_fold_scatter(FoldConsts C, const uint64_t* y, const int32_t* dst, uint64_t* x, int64_t items,
                               int nsl) {
  const int n = 1 << C.logn;
  const int64_t per = 2 * (int64_t)nsl * n;
  const int64_t total = items * per;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = e / per, w = e - u * per;
    x[(int64_t)dst[u] * per + w] = y[e];
  }
}

// ------------------------------------------------------------------ draws
// Key coefficients: for key kappa (column kappa * 8 + i), slot s of the key's slot list zm and digit
// i <= level: out[s][i][0][t] = uniform mod z (stream FKA, sub = stream id of z), out[s][i][1][t] =
// the Gaussian error (stream FKE, sub 0) as a residue mod z.
__global__ void k_fold_key_coeffs(FoldConsts C, uint64_t seed, int kappa, int level, SlotMap zm, const uint64_t* cdt,
                                  uint64_t* out) {
  const int n = 1 << C.logn;
  const int nsl = level + 2;
  const int64_t total = (int64_t)nsl * (level + 1) * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(e & (n - 1));
    const int64_t r = e >> C.logn;
    const int i = (int)(r % (level + 1));
    const int s = (int)(r / (level + 1));
    const int z = zm.z[s];
    const Mod md = C.mod[z];
    const uint64_t col = (uint64_t)kappa * 8 + (uint64_t)i;
    const uint64_t u = uniform_at(seed, stream_tag(kFKA, C.pid[z]), (uint64_t)t, col, md);
    const int32_t g = gaussian_at(seed, stream_tag(kFKE, 0), (uint64_t)t, col, cdt);
    out[(r * 2 + 0) * n + t] = u;
    out[(r * 2 + 1) * n + t] = from_signed(g, md.q, md.mu);
  }
}

// Key finish, NTT domain: beta = -k s + g_{s,i} s_from + e, stored as doubles [s][i][2][N]
// (part 0: k, part 1: beta).  s_hat, from_hat: [slot z][N] NTT residues; gk[s][i] = p (Q_l / q_i) mod z.
__global__ void k_fold_key_finish(FoldConsts C, int level, SlotMap zm, const uint64_t* coef_hat, const uint64_t* s_hat,
                                  const uint64_t* from_hat, KeyGadget gk, double* key) {
  const int n = 1 << C.logn;
  const int64_t total = (int64_t)(level + 2) * (level + 1) * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(e & (n - 1));
    const int64_t r = e >> C.logn;
    const int i = (int)(r % (level + 1));
    const int s = (int)(r / (level + 1));
    const int z = zm.z[s];
    const double zd = C.zd[z];
    const double k = to_d(coef_hat[(r * 2 + 0) * n + t]);
    const double err = to_d(coef_hat[(r * 2 + 1) * n + t]);
    double beta = submod_d(err, mm_d(k, to_d(s_hat[(int64_t)z * n + t]), z, C), zd);
    beta = addmod_d(beta, mm_d(gk.v[s][i], to_d(from_hat[(int64_t)z * n + t]), z, C), zd);
    key[(r * 2 + 0) * n + t] = k;
    key[(r * 2 + 1) * n + t] = beta;
  }
}

// Input errors: m[c][t] += the Gaussian at (t, c) of stream FXE.
__global__ void k_fold_add_errors(FoldConsts C, uint64_t seed, const uint64_t* cdt, int64_t* m, int64_t items) {
  const int n = 1 << C.logn;
  const int64_t total = items * (int64_t)n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e >> C.logn;
    const int t = (int)(e & (n - 1));
    m[e] += gaussian_at(seed, stream_tag(kFXE, 0), (uint64_t)t, (uint64_t)c, cdt);
  }
}

// Input masks and bodies, job = c * 5 + z: a (stream FXA, sub = stream id of q_z, element (t, c)) ->
// NTT -> ct[c][1][z]; ct[c][0][z] = (m + e)_hat - a_hat s_hat (the encoded inner products with their
// errors are already in ct[c][0][z]).
__global__ void __launch_bounds__(kNttThreads) k_fold_encrypt(FoldConsts C, uint64_t seed, const uint64_t* s_hat,
                                                            uint64_t* ct) {
  extern __shared__ double lds_raw[];
  const SwLds lds{lds_raw};
  const int n = 1 << C.logn;
  const int64_t c = blockIdx.x / 5;
  const int z = (int)(blockIdx.x - c * 5);
  const Mod md = C.mod[z];
  for (int t = threadIdx.x; t < n; t += blockDim.x)
    lds[t] = to_d(uniform_at(seed, stream_tag(kFXA, C.pid[z]), (uint64_t)t, (uint64_t)c, md));
  __syncthreads();
  ntt_fwd_lds(lds, C.tab[z]);
  uint64_t* b = ct + ((c * 2 + 0) * 5 + z) * n;
  uint64_t* a = ct + ((c * 2 + 1) * 5 + z) * n;
  const double zd = C.zd[z];
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const double av = lds[t];
    a[t] = to_u(av);
    b[t] = to_u(submod_d(to_d(b[t]), mm_d(av, to_d(s_hat[(int64_t)z * n + t]), z, C), zd));
  }
}

// Decryption at level 0 in the NTT domain: out[c][t] = b + a s mod q_0 (then an inverse transform).
__global__ void k_fold_dec_products(FoldConsts C, const uint64_t* ct, const uint64_t* s_hat, uint64_t* out,
                                    int64_t items) {
  const int n = 1 << C.logn;
  const int64_t total = items * (int64_t)n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e >> C.logn;
    const int t = (int)(e & (n - 1));
    const double b = to_d(ct[(c * 2 + 0) * n + t]), a = to_d(ct[(c * 2 + 1) * n + t]);
    out[e] = to_u(addmod_d(b, mm_d(a, to_d(s_hat[t]), 0, C), C.zd[0]));
  }
}

// Decoding (floating point), one workgroup per item: the slots m(zeta^(g_j)) of the centered coefficients
// m[c][0 .. N) as the DFT of length M of (m_i + i m_(M+i)) zeta^i (conjugate twiddles of the encoder's,
// bit-reversed input), real parts divided by the scale: v[c][j] at the transform's output k_j.
__global__ void __launch_bounds__(kNttThreads) k_fold_decode(const int64_t* m, int logn, const double* W,
                                                           const double* Z, const int32_t* kj, double inv_scale,
                                                           double* v) {
  extern __shared__ double lds[];
  const int M = 1 << (logn - 1);
  double* xr = lds;
  double* xi = lds + M;
  const int64_t c = blockIdx.x;
  const int64_t* mc = m + c * 2 * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const int p = (int)slot_brv((uint32_t)i, logn - 1);
    slot_twist((double)mc[i], (double)mc[M + i], Z[2 * i], Z[2 * i + 1], xr[p], xi[p]);
  }
  __syncthreads();
  for (int half = 1, lh = 0; half < M; half *= 2, ++lh) {
    const int step = M / (2 * half);
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int t = b & (half - 1);
      const int ia = ((b >> lh) << (lh + 1)) + t, ic = ia + half;
      slot_butterfly(xr[ia], xi[ia], xr[ic], xi[ic], W[2 * t * step], -W[2 * t * step + 1]);
    }
    __syncthreads();
  }
  for (int j = threadIdx.x; j < M; j += blockDim.x) v[c * M + j] = xr[kj[j]] * inv_scale;
}

unsigned ew_grid(int64_t total) {
  int64_t g = (total + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_fold_weights(const int32_t* values, int64_t total, int mode, int64_t* w, uint32_t* bad,
                               hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_weights, dim3(ew_grid(total)), dim3(256), 0, s, values, total, mode, w, bad);
  return hipGetLastError();
}

hipError_t launch_fold_encode(const int64_t* w, int64_t items, int logn, double scale, const double* W,
                              const double* Z, const int32_t* pos, int64_t* out, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << logn;
  hipError_t e = allow_lds(k_fold_encode, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold_encode, dim3((unsigned)items), dim3(ntt_block(logn)), lds, s, w, logn, scale, W, Z, pos,
                     out);
  return hipGetLastError();
}

hipError_t launch_fold_fwd(const FoldConsts& C, const int64_t* src, int64_t si, int64_t ss, uint64_t* dst, int64_t di,
                           int64_t ds, const SlotMap& zm, int nsl, int64_t items, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn;
  hipError_t e = allow_lds(k_fold_fwd, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold_fwd, dim3((unsigned)(items * nsl)), dim3(ntt_block(C.logn)), lds, s, C, src, si, ss, dst,
                     di, ds, zm, nsl);
  return hipGetLastError();
}

hipError_t launch_fold_inv(const FoldConsts& C, const FoldInv& a, int64_t items, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn;
  hipError_t e = allow_lds(k_fold_inv, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold_inv, dim3((unsigned)(items * a.nsl)), dim3(ntt_block(C.logn)), lds, s, C, a);
  return hipGetLastError();
}

hipError_t launch_fold_ks_mac(const FoldConsts& C, int level, const FoldInv& dg, const uint64_t* dig, const double* keys,
                              int64_t kstride, const int32_t* kidx, uint64_t* acc, int64_t* accp, int64_t items,
                              hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn;
  return by_regs(regs_per_thread(C.logn), [&](auto rc) -> hipError_t {
    constexpr int R = decltype(rc)::value;
    hipError_t e = allow_lds(k_fold_ks_mac<R>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold_ks_mac<R>, dim3((unsigned)(items * (level + 2))), dim3(ntt_block(C.logn)), lds, s, C,
                       level, dg, dig, keys, kstride, kidx, acc, accp);
    return hipGetLastError();
  });
}

hipError_t launch_fold_lift(const FoldConsts& C, const FoldLift& a, int64_t items, hipStream_t s) {
  if (items <= 0 || a.nsl <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn;
  hipError_t e = allow_lds(k_fold_lift, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold_lift, dim3((unsigned)(items * 2 * a.nsl)), dim3(ntt_block(C.logn)), lds, s, C, a);
  return hipGetLastError();
}

hipError_t launch_fold_relin_center(const FoldConsts& C, int level, const uint64_t* acc, const int64_t* accp,
                                   const uint64_t* tx, const uint64_t* ty, int64_t items, int64_t* cen, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn;
  hipError_t e = allow_lds(k_fold_relin_center, lds);
  if (e != hipSuccess) return e;
  const uint64_t ql = C.mod[level].q, p = C.mod[5].q;
  const double p_l = (double)(p % ql), pinv_l = (double)inv_mod(p % ql, ql);
  hipLaunchKernelGGL(k_fold_relin_center, dim3((unsigned)(items * 2)), dim3(ntt_block(C.logn)), lds, s, C, level, acc,
                     accp, tx, ty, p_l, pinv_l, (int64_t)(p * ql), cen);
  return hipGetLastError();
}

hipError_t launch_fold_perm(const FoldConsts& C, const uint64_t* x, const int32_t* src, const int32_t* amt,
                            const int32_t* perm, uint64_t* out, int64_t items, int nsl, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_perm, dim3(ew_grid(items * 2 * nsl << C.logn)), dim3(256), 0, s, C, x, src, amt, perm,
                     out, items, nsl);
  return hipGetLastError();
}

hipError_t launch_fold_group_sum(const FoldConsts& C, const uint64_t* f, const uint64_t* rotated, const int32_t* beg,
                                 const int32_t* mem, uint64_t* out, int64_t groups, int nsl, hipStream_t s) {
  if (groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_group_sum, dim3(ew_grid(groups * 2 * nsl << C.logn)), dim3(256), 0, s, C, f, rotated, beg,
                     mem, out, groups, nsl);
  return hipGetLastError();
}

hipError_t launch_fold_scatter(const FoldConsts& C, const uint64_t* y, const int32_t* dst, uint64_t* x, int64_t items,
                               int nsl, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_scatter, dim3(ew_grid(items * 2 * nsl << C.logn)), dim3(256), 0, s, C, y, dst, x, items,
                     nsl);
  return hipGetLastError();
}

hipError_t launch_fold_key_coeffs(const FoldConsts& C, uint64_t seed, int kappa, int level, const SlotMap& zm,
                                  const uint64_t* cdt, uint64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_key_coeffs, dim3(ew_grid((int64_t)(level + 2) * (level + 1) << C.logn)), dim3(256), 0, s,
                     C, seed, kappa, level, zm, cdt, out);
  return hipGetLastError();
}

hipError_t launch_fold_key_finish(const FoldConsts& C, int level, const SlotMap& zm, const uint64_t* coef_hat,
                                  const uint64_t* s_hat, const uint64_t* from_hat, const KeyGadget& gk, double* key,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_fold_key_finish, dim3(ew_grid((int64_t)(level + 2) * (level + 1) << C.logn)), dim3(256), 0, s,
                     C, level, zm, coef_hat, s_hat, from_hat, gk, key);
  return hipGetLastError();
}

hipError_t launch_fold_add_errors(const FoldConsts& C, uint64_t seed, const uint64_t* cdt, int64_t* m, int64_t items,
                                  hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_add_errors, dim3(ew_grid(items << C.logn)), dim3(256), 0, s, C, seed, cdt, m, items);
  return hipGetLastError();
}

hipError_t launch_fold_encrypt(const FoldConsts& C, uint64_t seed, const uint64_t* s_hat, uint64_t* ct, int64_t items,
                               hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << C.logn;
  hipError_t e = allow_lds(k_fold_encrypt, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold_encrypt, dim3((unsigned)(items * 5)), dim3(ntt_block(C.logn)), lds, s, C, seed, s_hat, ct);
  return hipGetLastError();
}

hipError_t launch_fold_dec_products(const FoldConsts& C, const uint64_t* ct, const uint64_t* s_hat, uint64_t* out,
                                    int64_t items, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_dec_products, dim3(ew_grid(items << C.logn)), dim3(256), 0, s, C, ct, s_hat, out, items);
  return hipGetLastError();
}

hipError_t launch_fold_decode(const int64_t* m, int64_t items, int logn, const double* W, const double* Z,
                              const int32_t* kj, double inv_scale, double* v, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const size_t lds = sizeof(double) << logn;
  hipError_t e = allow_lds(k_fold_decode, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fold_decode, dim3((unsigned)items), dim3(ntt_block(logn)), lds, s, m, logn, W, Z, kj,
                     inv_scale, v);
  return hipGetLastError();
}

}  // namespace hfe
