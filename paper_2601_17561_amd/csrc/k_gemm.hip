// The modular contraction of the CCMM (Section 2.3: the four plaintext matrix products, written
// as one product D X per prime; Section 6.3 reduces them to small-integer matrix products).
//
//   C[z][c][r] = sum_k D_z[src(r)][k] X_z[c][k]  mod prime_z
//
// for the prime slots z (the level's query primes, then p), query columns c < d3 and output
// rows r < R_out = N_DB + rows, where output rows map to database rows
// src(r) = r (A-part) for r < N_DB and N_DB + row0 + (r - N_DB) (the selected codes).
//
// Two forms, bit-identical results:
//  * plain: residues < 2^36 split into 18-bit limbs, limb products accumulated exactly in
//    64-bit integers on the vector ALU, one reduction per output;
//  * i8: centered residues split into 5 balanced int8 digits; the 25 digit-pair products run
//    on int8 MFMA (v_mfma_i32_32x32x32_i8) with the pairs of equal weight 256^(s+t) sharing
//    one int32 accumulator (9 accumulators), exact because a K-chunk of at most 32,704
//    keeps every partial sum below 2^31; recombination by Horner's rule in 64-bit integers
//    with a Barrett reduction at each step.
#include "hfe_device.h"

namespace hfe {

// ------------------------------------------------------------------ plain form
constexpr int kPR = 64;   // output rows per workgroup (one per lane)
constexpr int kPC = 32;   // query columns per workgroup (8 per wave)
constexpr int kPK = 16;   // K step

__global__ void __launch_bounds__(256) k_gemm_plain(GemmArgs g) {
  __shared__ uint2 sD[kPK][kPR];
  __shared__ uint2 sX[kPK][kPC];
  const int z = blockIdx.z;
  const uint64_t* __restrict__ Dt = g.Dt[z];
  const uint64_t* __restrict__ X = g.X[z];
  const int64_t r0 = (int64_t)blockIdx.x * kPR, c0 = (int64_t)blockIdx.y * kPC;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  // D loads: element e = tid + 256 i, kk = e / 64, rr = e % 64 -> rr = tx, kk = ty + 4 i
  const int64_t r_ld = r0 + tx;
  const bool r_ok = r_ld < g.R_out;
  const int64_t src = r_ok ? src_row(r_ld, g.n_db, g.row0) : 0;
  // X loads: e = tid + 256 i (i < 2), cc = e / 16, kk = e % 16
  const int kk_x = tid & 15;
  const int cc_x0 = tid >> 4, cc_x1 = (tid + 256) >> 4;
  uint64_t acc[8][3];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0;
  const uint32_t m18 = (1u << 18) - 1;
  for (int64_t k0 = 0; k0 < g.K; k0 += kPK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = ty + 4 * i;
      const int64_t k = k0 + kk;
      const uint64_t v = (r_ok && k < g.K) ? Dt[k * g.R_db + src] : 0;
      sD[kk][tx] = make_uint2((uint32_t)v & m18, (uint32_t)(v >> 18));
    }
    {
      const int64_t k = k0 + kk_x;
      const int64_t ca = c0 + cc_x0, cb = c0 + cc_x1;
      const uint64_t va = (ca < g.d3 && k < g.K) ? X[ca * g.K + k] : 0;
      const uint64_t vb = (cb < g.d3 && k < g.K) ? X[cb * g.K + k] : 0;
      sX[kk_x][cc_x0] = make_uint2((uint32_t)va & m18, (uint32_t)(va >> 18));
      sX[kk_x][cc_x1] = make_uint2((uint32_t)vb & m18, (uint32_t)(vb >> 18));
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kPK; ++kk) {
      const uint2 d = sD[kk][tx];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint2 x = sX[kk][ty * 8 + j];
        acc[j][0] += (uint64_t)d.x * x.x;
        acc[j][1] += (uint64_t)d.x * x.y + (uint64_t)d.y * x.x;
        acc[j][2] += (uint64_t)d.y * x.y;
      }
    }
    __syncthreads();
  }
  const Mod m = g.mod[z];
  const uint64_t c36 = barrett64(1ull << 36, m.q, m.mu);
  const uint64_t c36_sh = shoup_quot(c36, m.q);
  if (!r_ok) return;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t c = c0 + ty * 8 + j;
    if (c >= g.d3) continue;
    const uint64_t lo = barrett64(acc[j][0], m.q, m.mu);
    const uint64_t mid = barrett64(barrett64(acc[j][1], m.q, m.mu) << 18, m.q, m.mu);
    const uint64_t hi = mul_shoup(barrett64(acc[j][2], m.q, m.mu), c36, c36_sh, m.q);
    g.C[z][c * g.R_out + r_ld] = add_mod(add_mod(lo, mid, m.q), hi, m.q);
  }
}

hipError_t launch_gemm_plain(const GemmArgs& g, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.R_out + kPR - 1) / kPR), (unsigned)((g.d3 + kPC - 1) / kPC), (unsigned)g.nz);
  hipLaunchKernelGGL(k_gemm_plain, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ int8 MFMA form
constexpr int kLdsRow = 80;       // bytes per LDS row: 64 digits + 16 pad (conflict-free b128 reads)
constexpr int kChunkKB = 511;     // K-blocks per exact int32 chunk: 511 * 64 * 4 * 2^14 < 2^31

// Horner recombination of the 9 anti-diagonal sums a_u (weight 256^u) into a residue:
// r <- (r * 256 + a_u + q) mod q from u = 8 down to 0.  |a_u| < 2^31 < q, so every
// intermediate is in [0, 257 q + 2^31) < 2^45.
__device__ __forceinline__ uint64_t horner9(const int32_t a[9], uint64_t q, uint64_t mu) {
  uint64_t r = 0;
#pragma unroll
  for (int u = 8; u >= 0; --u) {
    const uint64_t x = (r << 8) + (uint64_t)((int64_t)a[u] + (int64_t)q);
    r = barrett64(x, q, mu);
  }
  return r;
}

// Tile schedule: the workgroups of one launch are dealt round-robin to the 8 XCDs (each with its
// own L2).  Workgroup i runs on XCD i % 8; tiles are numbered so that one XCD receives all
// query-column tiles of a database-row tile back to back, hence the database digits of that
// tile are fetched from HBM once into that XCD's L2 and shared by its query-column tiles.

// One output tile of one prime of one contraction problem.
struct I8Tile {
  const int8_t* Xd;   // query digits of this prime: [5][KB][d3_pad][64]
  const int8_t* Dd;   // database digits of this prime: [5][KB][R_pad][64]
  uint64_t* C;        // output of this prime: [d3][R_out]
  Mod m;
  int64_t KB, R_pad, d3_pad, n_db, row0, R_out, d3;
  int64_t r0, c0;     // tile origin: output row, query column
};

// Tile index within one prime of a problem -> (row tile, column tile), XCD-aware: tile index l
// runs on XCD l % 8 when the launch grid is a multiple of 8 and the problem starts at a
// multiple of 8.  Returns false for the padding tiles (row tile beyond the last one).
__device__ __forceinline__ bool tile_coords(int64_t l, int64_t n_rt, int64_t n_ct, int64_t& rt, int64_t& ct) {
  const int64_t xcd = l % kXcds, j = l / kXcds;
  rt = (j / n_ct) * kXcds + xcd;
  ct = j % n_ct;
  return rt < n_rt;
}

__device__ __forceinline__ void store_tile(const I8Tile& T, const v16i* acc, int wq, int wr, int lane, bool accumulate) {
  // 32x32 MFMA result layout: lane l, element j holds row (M = query) 8 (j / 4) + 4 (l / 32)
  // + j % 4 and column (N = database row) l % 32.
  const int64_t out_r = T.r0 + wr * 32 + (lane & 31);
  if (out_r >= T.R_out) return;
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    const int64_t c = T.c0 + wq * 32 + 8 * (jj >> 2) + 4 * (lane >> 5) + (jj & 3);
    if (c >= T.d3) continue;
    int32_t a9[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) a9[u] = acc[u][jj];
    uint64_t v = horner9(a9, T.m.q, T.m.mu);
    uint64_t* dst = T.C + c * T.R_out + out_r;
    if (accumulate) v = add_mod(v, *dst, T.m.q);
    *dst = v;
  }
}

// Workgroup tile: WR x WQ waves, each owning a 32 (query) x 32 (database row) block of the
// output; NBUF LDS stages (1: load, barrier, compute, barrier; 2: compute one stage while the
// next is written).  lds: NBUF * 5 * (32 WQ + 32 WR) * kLdsRow bytes.
template <int WR, int WQ, int NBUF>
__device__ __forceinline__ void tile_basic(const I8Tile& T, int8_t* lds) {
  constexpr int NT = 64 * WR * WQ;
  constexpr int BR = 32 * WR, BQ = 32 * WQ;
  constexpr int LA = (BQ * 4 + NT - 1) / NT;  // 16-byte loads per thread per query digit plane
  constexpr int LB = (BR * 4 + NT - 1) / NT;  // ... per database digit plane
  auto sA = [&](int buf, int t) { return lds + ((size_t)(buf * kDigits + t) * BQ) * kLdsRow; };
  auto sB = [&](int buf, int t) {
    return lds + (size_t)NBUF * kDigits * BQ * kLdsRow + ((size_t)(buf * kDigits + t) * BR) * kLdsRow;
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave % WQ, wr = wave / WQ;
  const size_t planeB = (size_t)T.KB * T.R_pad * kKB, planeA = (size_t)T.KB * T.d3_pad * kKB;
  const size_t stepB = (size_t)T.R_pad * kKB, stepA = (size_t)T.d3_pad * kKB;
  // global -> LDS: load i of a plane covers 16 bytes (chunk idx & 3) of tile row idx >> 2,
  // idx = tid + i NT.  Database rows map to source rows (< R_pad, zero padding); query columns
  // stay below d3_pad.
  const int8_t* gA[LA];
  const int8_t* gB[LB];
  bool okA[LA], okB[LB];
  int offA[LA], offB[LB];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int idx = tid + i * NT;
    okA[i] = idx < BQ * 4;
    const int row = okA[i] ? idx >> 2 : 0, ch = idx & 3;
    gA[i] = T.Xd + (size_t)(T.c0 + row) * kKB + ch * 16;
    offA[i] = row * kLdsRow + ch * 16;
  }
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    const int idx = tid + i * NT;
    okB[i] = idx < BR * 4;
    const int row = okB[i] ? idx >> 2 : 0, ch = idx & 3;
    gB[i] = T.Dd + (size_t)src_row(T.r0 + row, T.n_db, T.row0) * kKB + ch * 16;
    offB[i] = row * kLdsRow + ch * 16;
  }
  v4i pa[kDigits][LA], pb[kDigits][LB];
  auto fetch = [&](int64_t kb) {
#pragma unroll
    for (int t = 0; t < kDigits; ++t) {
#pragma unroll
      for (int i = 0; i < LA; ++i)
        if (okA[i]) pa[t][i] = *reinterpret_cast<const v4i*>(gA[i] + t * planeA + kb * stepA);
#pragma unroll
      for (int i = 0; i < LB; ++i)
        if (okB[i]) pb[t][i] = *reinterpret_cast<const v4i*>(gB[i] + t * planeB + kb * stepB);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kDigits; ++t) {
#pragma unroll
      for (int i = 0; i < LA; ++i)
        if (okA[i]) *reinterpret_cast<v4i*>(sA(buf, t) + offA[i]) = pa[t][i];
#pragma unroll
      for (int i = 0; i < LB; ++i)
        if (okB[i]) *reinterpret_cast<v4i*>(sB(buf, t) + offB[i]) = pb[t][i];
    }
  };
  for (int64_t kb0 = 0; kb0 < T.KB; kb0 += kChunkKB) {
    const int64_t kb1 = kb0 + kChunkKB < T.KB ? kb0 + kChunkKB : T.KB;
    v16i acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    fetch(kb0);
    if (NBUF == 2) {
      stash(0);
      __syncthreads();
    }
    for (int64_t kb = kb0; kb < kb1; ++kb) {
      const int cur = NBUF == 2 ? (int)((kb - kb0) & 1) : 0;
      const bool more = kb + 1 < kb1;
      if (NBUF == 1) {
        stash(0);
        __syncthreads();
      }
      if (more) fetch(kb + 1);
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int koff = half * 32 + (lane >> 5) * 16;
        v4i a[kDigits];
#pragma unroll
        for (int t = 0; t < kDigits; ++t)
          a[t] = *reinterpret_cast<const v4i*>(sA(cur, t) + (wq * 32 + (lane & 31)) * kLdsRow + koff);
#pragma unroll
        for (int s = 0; s < kDigits; ++s) {
          const v4i b = *reinterpret_cast<const v4i*>(sB(cur, s) + (wr * 32 + (lane & 31)) * kLdsRow + koff);
#pragma unroll
          for (int t = 0; t < kDigits; ++t)
            acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[t], b, acc[s + t], 0, 0, 0);
        }
      }
      if (NBUF == 2 && more) stash(cur ^ 1);
      __syncthreads();
    }
    store_tile(T, acc, wq, wr, lane, kb0 != 0);
  }
}

// Software-pipelined tile (2 x 2 waves, 64 x 64): two register sets carry K-blocks i + 1 and
// i + 2 while block i is multiplied from LDS, and the LDS stores of block i + 1 are issued
// between the MFMAs of block i, so that stores, global loads and the one barrier per block
// overlap the matrix pipe.  lds: 2 * 5 * 128 * kLdsRow bytes.
__device__ __forceinline__ void tile_pipe(const I8Tile& T, int8_t* lds) {
  constexpr int BR = 64, BQ = 64;
  constexpr int planeA_l = BQ * kLdsRow, planeB_l = BR * kLdsRow;
  auto sA = [&](int buf, int t) { return lds + ((size_t)(buf * kDigits + t) * BQ) * kLdsRow; };
  auto sB = [&](int buf, int t) {
    return lds + (size_t)2 * kDigits * BQ * kLdsRow + ((size_t)(buf * kDigits + t) * BR) * kLdsRow;
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave & 1, wr = wave >> 1;
  const size_t planeB = (size_t)T.KB * T.R_pad * kKB, planeA = (size_t)T.KB * T.d3_pad * kKB;
  const size_t stepB = (size_t)T.R_pad * kKB, stepA = (size_t)T.d3_pad * kKB;
  const int ld_row = tid >> 2, ld_ch = tid & 3;
  const int8_t* gA = T.Xd + (size_t)(T.c0 + ld_row) * kKB + ld_ch * 16;
  const int8_t* gB = T.Dd + (size_t)src_row(T.r0 + ld_row, T.n_db, T.row0) * kKB + ld_ch * 16;
  const int st_off = ld_row * kLdsRow + ld_ch * 16;
  const int rd_a = (wq * 32 + (lane & 31)) * kLdsRow, rd_b = (wr * 32 + (lane & 31)) * kLdsRow;

  v4i p0[2 * kDigits], p1[2 * kDigits];  // [A digits 0..4, B digits 0..4] of one K-block
  auto fetch = [&](v4i* p, int64_t kb) {
#pragma unroll
    for (int t = 0; t < kDigits; ++t) {
      p[t] = *reinterpret_cast<const v4i*>(gA + t * planeA + kb * stepA);
      p[kDigits + t] = *reinterpret_cast<const v4i*>(gB + t * planeB + kb * stepB);
    }
  };
  auto put = [&](const v4i* p, int buf, int i) {  // i-th of the 10 16-byte stores of a block
    if (i < kDigits)
      *reinterpret_cast<v4i*>(sA(buf, i) + st_off) = p[i];
    else
      *reinterpret_cast<v4i*>(sB(buf, i - kDigits) + st_off) = p[i];
  };

  for (int64_t kb0 = 0; kb0 < T.KB; kb0 += kChunkKB) {
    const int64_t kb_end = kb0 + kChunkKB < T.KB ? kb0 + kChunkKB : T.KB;
    const int64_t n = kb_end - kb0;
    v16i acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    fetch(p0, kb0);
#pragma unroll
    for (int i = 0; i < 2 * kDigits; ++i) put(p0, 0, i);
    fetch(p1, n > 1 ? kb0 + 1 : kb0);
    __syncthreads();
    // One K-block: multiply LDS stage `cur`; store the next block (register set `nx`) into the
    // other stage between the MFMAs (a store past the last block is harmless: that stage is
    // not read again); the block after next is loaded into set `ld` first (clamped to the last
    // block, so every load is in range and the code has no data-dependent branches).
    // Fragments are read one step ahead so LDS latency overlaps the MFMAs.
    auto block = [&](int cur, v4i* nx, v4i* ld, int64_t i) {
      fetch(ld, kb0 + i + 2 < kb_end ? kb0 + i + 2 : kb_end - 1);
      __builtin_amdgcn_sched_barrier(0);  // keep the global loads at the head of the block
      const int8_t* A = sA(cur, 0) + rd_a;
      const int8_t* B = sB(cur, 0) + rd_b;
      const int k0 = (lane >> 5) * 16, k1 = 32 + (lane >> 5) * 16;
      v4i a0[kDigits], a1[kDigits], b_cur, b_nxt;
#pragma unroll
      for (int t = 0; t < kDigits; ++t) a0[t] = *reinterpret_cast<const v4i*>(A + t * planeA_l + k0);
      b_cur = *reinterpret_cast<const v4i*>(B + k0);
#pragma unroll
      for (int step = 0; step < 2 * kDigits; ++step) {
        const int half = step / kDigits, s = step % kDigits;
        if (step + 1 < 2 * kDigits) {
          const int hs = (step + 1) / kDigits, ss = (step + 1) % kDigits;
          b_nxt = *reinterpret_cast<const v4i*>(B + ss * planeB_l + (hs ? k1 : k0));
        }
        if (step < kDigits) a1[step] = *reinterpret_cast<const v4i*>(A + step * planeA_l + k1);
        put(nx, cur ^ 1, step);
#pragma unroll
        for (int t = 0; t < kDigits; ++t)
          acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(half ? a1[t] : a0[t], b_cur, acc[s + t], 0, 0, 0);
        b_cur = b_nxt;
      }
      __syncthreads();
    };
    for (int64_t i = 0; i < n; i += 2) {
      block(0, p1, p0, i);
      if (i + 1 < n) block(1, p0, p1, i + 1);
    }
    store_tile(T, acc, wq, wr, lane, kb0 != 0);
  }
}

// Tile fed by direct global-to-LDS loads (global_load_lds_dwordx4: each lane's 16 bytes land
// at M0 + 16 * lane, so one instruction of a wave fills 16 rows of 64 bytes), STAGES LDS stages,
// so later K-blocks are in flight while block i is multiplied and no registers stage the data.
// WR x WQ waves, each owning a 32 (query) x 32 (database row) output block.  Rows are 64 bytes
// without padding; the 16-byte chunk c of row r sits at chunk position c ^ ((r >> 2) & 3), which
// makes the b128 fragment reads of 16 consecutive rows hit 64 distinct banks.  Wait counts are
// managed here: with three stages every wave issues the same number of loads per block and waits
// until only the next block's are outstanding, with two stages it waits for all.
// lds: STAGES x 5 x (32 WQ + 32 WR) rows x 64 bytes.
constexpr int kDmaRow = kKB;  // LDS bytes per tile row


template <int WR, int WQ, int STAGES>
__device__ __forceinline__ void tile_dma(const I8Tile& T, int8_t* lds) {
  constexpr int NW = WR * WQ, BR = 32 * WR, BQ = 32 * WQ;
  constexpr int kPA = BQ * kDmaRow, kPB = BR * kDmaRow, kStage = kDigits * (kPA + kPB);
  constexpr int LA = (BQ / 16 + NW - 1) / NW, LB = (BR / 16 + NW - 1) / NW;  // loads per wave per plane
  static_assert(STAGES == 2 || (STAGES == 3 && BQ / 16 % NW == 0 && BR / 16 % NW == 0),
                "three stages need the same load count on every wave");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave % WQ, wr = wave / WQ;
  const size_t planeB = (size_t)T.KB * T.R_pad * kKB, planeA = (size_t)T.KB * T.d3_pad * kKB;
  const size_t stepB = (size_t)T.R_pad * kKB, stepA = (size_t)T.d3_pad * kKB;
  // load j of a wave fills plane rows 16 (wave + NW j) .. + 15: lane l -> row + l / 4, stored
  // chunk l % 4, which holds logical chunk (l % 4) ^ ((row >> 2) & 3) (the same for every j,
  // since 16 NW j is a multiple of 16)
  const int ld_row = 16 * wave + (lane >> 2);
  const int ld_chunk = ((lane & 3) ^ ((ld_row >> 2) & 3)) * 16;
  const int8_t* gA[LA];
  const int8_t* gB[LB];
#pragma unroll
  for (int j = 0; j < LA; ++j) gA[j] = T.Xd + (size_t)(T.c0 + ld_row + 16 * NW * j) * kKB + ld_chunk;
#pragma unroll
  for (int j = 0; j < LB; ++j)
    gB[j] = T.Dd + (size_t)src_row(T.r0 + ld_row + 16 * NW * j, T.n_db, T.row0) * kKB + ld_chunk;
  const uint32_t lds0 = (uint32_t)(uintptr_t)lds + wave * 16 * kDmaRow;
  auto issue = [&](int stage, int64_t kb) {
    const uint32_t base = lds0 + stage * kStage;
#pragma unroll
    for (int t = 0; t < kDigits; ++t) {
#pragma unroll
      for (int j = 0; j < LA; ++j)
        if (16 * (wave + NW * j) < BQ) dma16(gA[j] + t * planeA + kb * stepA, base + t * kPA + 16 * NW * j * kDmaRow);
#pragma unroll
      for (int j = 0; j < LB; ++j)
        if (16 * (wave + NW * j) < BR)
          dma16(gB[j] + t * planeB + kb * stepB, base + kDigits * kPA + t * kPB + 16 * NW * j * kDmaRow);
    }
  };
  // fragment reads: row r, logical chunk c -> byte r * 64 + ((c ^ ((r >> 2) & 3)) * 16); the
  // query row wq 32 + l % 32 and database row wr 32 + l % 32 share the swizzle
  const int sw = ((lane & 31) >> 2) & 3;
  const int offA = (wq * 32 + (lane & 31)) * kDmaRow, offB = kDigits * kPA + (wr * 32 + (lane & 31)) * kDmaRow;
  const int c0 = lane >> 5;  // logical chunk of the first K-half; the second half adds 2

  for (int64_t kb0 = 0; kb0 < T.KB; kb0 += kChunkKB) {
    const int64_t kb_end = kb0 + kChunkKB < T.KB ? kb0 + kChunkKB : T.KB;
    const int64_t n = kb_end - kb0;
    auto clamp = [&](int64_t i) { return kb0 + (i < n ? i : n - 1); };
    v16i acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < STAGES - 1; ++j) issue(j, clamp(j));
    for (int64_t i = 0; i < n; ++i) {
      const int st = (int)(i % STAGES);
      // block i complete for this wave (with three stages block i + 1 may still fly), then for
      // all waves; all waves are also done reading the stage that block i + STAGES - 1 overwrites
      if constexpr (STAGES == 3) {
        static_assert(kDigits * (BQ / 16 / NW + BR / 16 / NW) == 10, "vmcnt below assumes 10 loads per block");
        asm volatile("s_waitcnt vmcnt(10) lgkmcnt(0)\n\ts_barrier" ::: "memory");
      } else {
        asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
      }
      issue((int)((i + STAGES - 1) % STAGES), clamp(i + STAGES - 1));
      const int8_t* S = lds + st * kStage;
      auto fa = [&](int t, int c) { return *reinterpret_cast<const v4i*>(S + offA + t * kPA + ((c ^ sw) << 4)); };
      auto fb = [&](int t, int c) { return *reinterpret_cast<const v4i*>(S + offB + t * kPB + ((c ^ sw) << 4)); };
      v4i a0[kDigits], a1[kDigits], b_cur, b_nxt;
#pragma unroll
      for (int t = 0; t < kDigits; ++t) a0[t] = fa(t, c0);
      b_cur = fb(0, c0);
#pragma unroll
      for (int step = 0; step < 2 * kDigits; ++step) {
        const int half = step / kDigits, s = step % kDigits;
        if (step + 1 < 2 * kDigits) b_nxt = fb((step + 1) % kDigits, c0 + 2 * ((step + 1) / kDigits));
        if (step < kDigits) a1[step] = fa(step, c0 + 2);
#pragma unroll
        for (int t = 0; t < kDigits; ++t)
          acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(half ? a1[t] : a0[t], b_cur, acc[s + t], 0, 0, 0);
        b_cur = b_nxt;
      }
    }
    // drain the clamped loads still in flight before the stages are reused
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    store_tile(T, acc, wq, wr, lane, kb0 != 0);
  }
}

// DMA-fed tile with separate LDS rings for the two operands: the database digits (streamed from
// HBM once per launch, so their loads see the longest latency) in three stages, loaded two K-blocks
// ahead, and the query digits (re-read by every database-row tile, mostly from L2) in two stages,
// loaded one block ahead.  Both rings fit where three stages of both would not (64 x 128: 2 x 40 +
// 3 x 20 KiB).  Per block, wave w issues its query loads and then its database loads; at the barrier
// of block i it waits until only its database loads of block i + 1 are outstanding (vmcnt counts
// them in issue order).  Loads are dealt to waves round-robin: query load j (plane j / nQ, row
// group j % nQ) to wave j % NW, database load j likewise, so waves differ in their database load
// count and each waits for its own.  Fragment reads, swizzle and MFMA order as tile_dma.
template <int WR, int WQ>
__device__ __forceinline__ void tile_dma_split(const I8Tile& T, int8_t* lds) {
  constexpr int NW = WR * WQ, BR = 32 * WR, BQ = 32 * WQ;
  constexpr int nQ = BQ / 16, nB = BR / 16;                  // 16-row groups per plane
  constexpr int kPA = BQ * kDmaRow, kPB = BR * kDmaRow;      // bytes per plane
  constexpr int kQS = kDigits * kPA, kBS = kDigits * kPB;    // bytes per stage
  constexpr int LQ = (kDigits * nQ + NW - 1) / NW, LB = (kDigits * nB + NW - 1) / NW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave % WQ, wr = wave / WQ;
  const size_t planeB = (size_t)T.KB * T.R_pad * kKB, planeA = (size_t)T.KB * T.d3_pad * kKB;
  const size_t stepB = (size_t)T.R_pad * kKB, stepA = (size_t)T.d3_pad * kKB;
  // lane l of a load covers row 16 g + l / 4, stored chunk l % 4 = logical chunk
  // (l % 4) ^ ((row >> 2) & 3) = (l % 4) ^ ((l >> 4) & 3)
  const int lrow = lane >> 2, lchunk = ((lane & 3) ^ ((lane >> 4) & 3)) * 16;
  const int8_t* gq[LQ];
  const int8_t* gb[LB];
  uint32_t oq[LQ], ob[LB];
  bool vq[LQ], vb[LB];
  int cb = 0;  // this wave's database loads per block
#pragma unroll
  for (int j = 0; j < LQ; ++j) {
    const int i = wave + NW * j;
    vq[j] = i < kDigits * nQ;
    const int t = vq[j] ? i / nQ : 0, g = vq[j] ? i % nQ : 0;
    gq[j] = T.Xd + t * planeA + (size_t)(T.c0 + 16 * g + lrow) * kKB + lchunk;
    oq[j] = t * kPA + 16 * g * kDmaRow;
  }
#pragma unroll
  for (int j = 0; j < LB; ++j) {
    const int i = wave + NW * j;
    vb[j] = i < kDigits * nB;
    cb += vb[j] ? 1 : 0;
    const int t = vb[j] ? i / nB : 0, g = vb[j] ? i % nB : 0;
    gb[j] = T.Dd + t * planeB + (size_t)src_row(T.r0 + 16 * g + lrow, T.n_db, T.row0) * kKB + lchunk;
    ob[j] = 2 * kQS + t * kPB + 16 * g * kDmaRow;
  }
  const uint32_t lds0 = (uint32_t)(uintptr_t)lds;
  auto issue_q = [&](int stage, int64_t kb) {
#pragma unroll
    for (int j = 0; j < LQ; ++j)
      if (vq[j]) dma16(gq[j] + kb * stepA, lds0 + stage * kQS + oq[j]);
  };
  auto issue_b = [&](int stage, int64_t kb) {
#pragma unroll
    for (int j = 0; j < LB; ++j)
      if (vb[j]) dma16(gb[j] + kb * stepB, lds0 + stage * kBS + ob[j]);
  };
  // wait until at most this wave's database loads of one block are outstanding, then barrier
  auto wait_barrier = [&]() {
    static_assert(LB <= 5, "the waits below cover up to five database loads per wave and block");
    if (cb >= 5) asm volatile("s_waitcnt vmcnt(5)" ::: "memory");
    else if (cb == 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    else if (cb == 3) asm volatile("s_waitcnt vmcnt(3)" ::: "memory");
    else if (cb == 2) asm volatile("s_waitcnt vmcnt(2)" ::: "memory");
    else if (cb == 1) asm volatile("s_waitcnt vmcnt(1)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  };
  const int sw = ((lane & 31) >> 2) & 3;
  const int offA = (wq * 32 + (lane & 31)) * kDmaRow, offB = 2 * kQS + (wr * 32 + (lane & 31)) * kDmaRow;
  const int c0 = lane >> 5;

  for (int64_t kb0 = 0; kb0 < T.KB; kb0 += kChunkKB) {
    const int64_t kb_end = kb0 + kChunkKB < T.KB ? kb0 + kChunkKB : T.KB;
    const int64_t n = kb_end - kb0;
    auto clamp = [&](int64_t i) { return kb0 + (i < n ? i : n - 1); };
    v16i acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    issue_b(0, clamp(0));
    issue_q(0, clamp(0));
    issue_b(1, clamp(1));
    for (int64_t i = 0; i < n; ++i) {
      // block i (query loads issued at i - 1, database loads at i - 2) complete for every wave,
      // and every wave is done with block i - 1, whose stages the loads below overwrite
      wait_barrier();
      issue_q((int)((i + 1) & 1), clamp(i + 1));
      issue_b((int)((i + 2) % 3), clamp(i + 2));
      const int8_t* SA = lds + (i & 1) * kQS;
      const int8_t* SB = lds + (i % 3) * kBS;
      auto fa = [&](int t, int c) { return *reinterpret_cast<const v4i*>(SA + offA + t * kPA + ((c ^ sw) << 4)); };
      auto fb = [&](int t, int c) { return *reinterpret_cast<const v4i*>(SB + offB + t * kPB + ((c ^ sw) << 4)); };
      v4i a0[kDigits], a1[kDigits], b_cur, b_nxt;
#pragma unroll
      for (int t = 0; t < kDigits; ++t) a0[t] = fa(t, c0);
      b_cur = fb(0, c0);
#pragma unroll
      for (int step = 0; step < 2 * kDigits; ++step) {
        const int half = step / kDigits, s = step % kDigits;
        if (step + 1 < 2 * kDigits) b_nxt = fb((step + 1) % kDigits, c0 + 2 * ((step + 1) / kDigits));
        if (step < kDigits) a1[step] = fa(step, c0 + 2);
#pragma unroll
        for (int t = 0; t < kDigits; ++t)
          acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(half ? a1[t] : a0[t], b_cur, acc[s + t], 0, 0, 0);
        b_cur = b_nxt;
      }
    }
    // drain the clamped loads still in flight before the stages are reused
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    store_tile(T, acc, wq, wr, lane, kb0 != 0);
  }
}

// Grid launch: blockIdx.z = prime slot, blockIdx.x = XCD-ordered tile.
template <int WR, int WQ, int NBUF, int WPE, int MODE>
constexpr int lds_bytes() {
  if constexpr (MODE == 3) return kDigits * (2 * 32 * WQ + 3 * 32 * WR) * kDmaRow;  // 2 query + 3 database stages
  return NBUF * kDigits * (32 * WQ + 32 * WR) * (MODE == 2 ? kDmaRow : kLdsRow);
}

template <int WR, int WQ, int NBUF, int WPE, int MODE>
__device__ __forceinline__ void run_tile(const I8Tile& T, int8_t* lds) {
  if constexpr (MODE == 3)
    tile_dma_split<WR, WQ>(T, lds);
  else if constexpr (MODE == 2)
    tile_dma<WR, WQ, NBUF>(T, lds);
  else if constexpr (MODE == 1)
    tile_pipe(T, lds);
  else
    tile_basic<WR, WQ, NBUF>(T, lds);
}

template <int WR, int WQ, int NBUF, int WPE, int MODE>
__global__ void __launch_bounds__(64 * WR * WQ) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_gemm_i8(GemmArgs g) {
  constexpr int BR = 32 * WR, BQ = 32 * WQ;
  __shared__ __attribute__((aligned(16))) int8_t lds[lds_bytes<WR, WQ, NBUF, WPE, MODE>()];
  const int z = blockIdx.z;
  const int64_t n_ct = (g.d3 + BQ - 1) / BQ, n_rt = (g.R_out + BR - 1) / BR;
  int64_t rt, ct;
  if (!tile_coords(blockIdx.x, n_rt, n_ct, rt, ct)) return;
  I8Tile T{g.Xd[z], g.Dd[z], g.C[z], g.mod[z], g.KB, g.R_pad, g.d3_pad, g.n_db, g.row0, g.R_out, g.d3,
           rt * BR, ct * BQ};
  run_tile<WR, WQ, NBUF, WPE, MODE>(T, lds);
}

// Persistent grouped launch over a table of problems (batched CCMM): workgroup w processes
// tiles w, w + G, w + 2G, ... of the concatenated tile list (G = grid size, a multiple of 8,
// and every problem starts at a multiple of 8, so tile t always runs on XCD t % 8).
template <int WR, int WQ, int NBUF, int WPE, int MODE>
__global__ void __launch_bounds__(64 * WR * WQ) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_gemm_i8_batched(BatchGemmArgs a) {
  constexpr int BR = 32 * WR, BQ = 32 * WQ;
  // no other LDS than the tile's, so that the tile's occupancy holds
  __shared__ __attribute__((aligned(16))) int8_t lds[lds_bytes<WR, WQ, NBUF, WPE, MODE>()];
  const int n = a.hdr->n;
  // Tiles are claimed in order from one counter per XCD (workgroup b runs on XCD b mod 8), so
  // the workgroups of an XCD always work on a contiguous window of tiles that share database
  // and query blocks in L2, however unevenly tiles finish; tile t = 8 j + xcd.  The claim is
  // passed to the workgroup through the first LDS word, which no tile uses between tiles.
  const int xcd = blockIdx.x % kXcds;
  const int64_t per_xcd = a.hdr->total_tiles / kXcds;
  for (;;) {
    __syncthreads();  // the previous tile is done with LDS
    if (threadIdx.x == 0) *reinterpret_cast<uint32_t*>(lds) = atomicAdd(a.next + xcd, 1u);
    __syncthreads();
    // uniform by construction; readfirstlane tells the compiler, so that the descriptor and
    // tile coordinates below live in scalar registers as kernel arguments do
    const int64_t j = (uint32_t)__builtin_amdgcn_readfirstlane(*reinterpret_cast<const uint32_t*>(lds));
    __syncthreads();  // every thread has read the claim before the tile overwrites LDS
    if (j >= per_xcd) break;
    const int64_t t = j * kXcds + xcd;
    int lo = 0, hi = n - 1;  // last problem whose first tile is <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.desc[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const BatchDesc& d = a.desc[lo];
    const int64_t n_ct = (d.d3 + BQ - 1) / BQ, n_rt = (d.R_out + BR - 1) / BR;
    const int64_t per_prime = (n_rt + kXcds - 1) / kXcds * kXcds * n_ct;
    const int64_t local = t - d.tile_begin;
    const int z = (int)(local / per_prime);
    int64_t rt, ct;
    if (!tile_coords(local % per_prime, n_rt, n_ct, rt, ct)) continue;
    const size_t planeX = (size_t)a.KB * d.d3_pad * kKB * kDigits;
    const size_t planeD = (size_t)a.KB * a.R_pad * kKB * kDigits;
    I8Tile T{d.Xd + z * planeX, a.Dd + d.slot[z] * planeD, d.C + (size_t)z * d.d3 * d.R_out, d.mod[z], a.KB,
             a.R_pad, d.d3_pad, d.n_db, d.row0, d.R_out, d.d3, rt * BR, ct * BQ};
    run_tile<WR, WQ, NBUF, WPE, MODE>(T, lds);
  }
}

struct I8Variant {
  const char* name;
  void (*grid)(GemmArgs);
  void (*batched)(BatchGemmArgs);
  int br, bq, threads, waves_per_simd;
};

#define HFE_I8_VARIANT(NAME, WR, WQ, NB, WPE, MODE)                                                          \
  {                                                                                                          \
    NAME, k_gemm_i8<WR, WQ, NB, WPE, MODE>, k_gemm_i8_batched<WR, WQ, NB, WPE, MODE>, 32 * (WR), 32 * (WQ), \
        64 * (WR) * (WQ), (WPE)                                                                              \
  }

// MODE 0: tile_basic, 1: tile_pipe, 2: tile_dma (NB = LDS stages), 3: tile_dma_split.  The first
// entry is the default.
static const I8Variant kI8Variants[] = {
    HFE_I8_VARIANT("dma_r128_w2", 4, 2, 2, 2, 2), HFE_I8_VARIANT("dma_q128_w2", 2, 4, 2, 2, 2),
    HFE_I8_VARIANT("dmas_q128_w2", 2, 4, 0, 2, 3), HFE_I8_VARIANT("dmas_r128_w2", 4, 2, 0, 2, 3),
    HFE_I8_VARIANT("dma2_w2", 2, 2, 2, 2, 2),     HFE_I8_VARIANT("dma3_w1", 2, 2, 3, 1, 2),
    HFE_I8_VARIANT("pipe_w1", 2, 2, 2, 1, 1),
    HFE_I8_VARIANT("r2q2b1w1", 2, 2, 1, 1, 0),    HFE_I8_VARIANT("r2q2b2w1", 2, 2, 2, 1, 0),
    HFE_I8_VARIANT("r2q2b1w2", 2, 2, 1, 2, 0),    HFE_I8_VARIANT("r4q2b1w2", 4, 2, 1, 2, 0),
    HFE_I8_VARIANT("r2q4b1w2", 2, 4, 1, 2, 0),
};
constexpr int kNumI8Variants = sizeof(kI8Variants) / sizeof(kI8Variants[0]);
static_assert(kNumI8Variants <= kMaxI8Variants, "raise kMaxI8Variants");

int i8_variant_count() { return kNumI8Variants; }
const char* i8_variant_name(int v) { return (v >= 0 && v < kNumI8Variants) ? kI8Variants[v].name : nullptr; }
int i8_variant_tile_rows(int v) { return kI8Variants[v].br; }
int i8_variant_tile_cols(int v) { return kI8Variants[v].bq; }
int i8_variant_wgs_per_cu(int v) { return kI8Variants[v].waves_per_simd * 4 * 64 / kI8Variants[v].threads; }

hipError_t launch_gemm_i8(const GemmArgs& g, int variant, hipStream_t s) {
  if (g.R_out <= 0 || g.d3 <= 0) return hipSuccess;
  if (variant < 0 || variant >= kNumI8Variants) return hipErrorInvalidValue;
  const I8Variant& v = kI8Variants[variant];
  if (g.d3_pad % v.bq != 0) return hipErrorInvalidValue;  // query padding must cover the tile
  const int64_t n_ct = (g.d3 + v.bq - 1) / v.bq, n_rt = (g.R_out + v.br - 1) / v.br;
  const int64_t n_rt8 = (n_rt + kXcds - 1) / kXcds * kXcds;
  dim3 grid((unsigned)(n_rt8 * n_ct), 1, (unsigned)g.nz);
  hipLaunchKernelGGL(v.grid, grid, dim3(v.threads), 0, s, g);
  return hipGetLastError();
}

int64_t i8_batched_tiles(int variant, int64_t d3, int64_t R_out, int nz) {
  const I8Variant& v = kI8Variants[variant];
  const int64_t n_ct = (d3 + v.bq - 1) / v.bq, n_rt = (R_out + v.br - 1) / v.br;
  return (n_rt + kXcds - 1) / kXcds * kXcds * n_ct * nz;
}

hipError_t launch_gemm_i8_batched(const BatchGemmArgs& a, int variant, int grid, hipStream_t s) {
  if (variant < 0 || variant >= kNumI8Variants) return hipErrorInvalidValue;
  const I8Variant& v = kI8Variants[variant];
  hipLaunchKernelGGL(v.batched, dim3((unsigned)grid), dim3(v.threads), 0, s, a);
  return hipGetLastError();
}

}  // namespace hfe
