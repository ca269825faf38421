"""Counter-based randomness and samplers (oracle).

The paper fixes no random generator (it defers key generation and encryption
to the CKKS literature), yet bit-exact agreement of two independent
implementations needs one.  Both sides therefore implement the same published
counter-based generator, Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011), and the same stream layout:

  key     = (seed, purpose << 32 | sub)
  counter = (c0, c1, c2, c3), one 4 x 64-bit block per counter value

  purpose  sub        element index (i0, i1)     distribution
  1 QSEC   chunk j    (coef t, 0)                ternary  (query secret s_j)
  2 DBSEC  chunk j    (coef t, 0)                ternary  (database secret s'_j)
  3 DBA    prime id   (coef v < N_DB, column c)  uniform mod prime (A1 | A2)
  4 DBE    0          (db row i, column c)       Gaussian (E1 | E2)
  5 QA     prime id   (coef t < N_Q, column c)   uniform mod prime (a_c)
  6 QE     0          (code row t, column c)     Gaussian (e_c)

  prime id: i for query prime q_i, 16 for the special prime p.

Samplers (element (i0, i1)):
  uniform mod q / ternary (q = 3, value - 1):
      w = philox(key, (i0 >> 2, i1, 0, 0))[i0 & 3]; accept if w < floor(2^64/q)*q,
      value = w mod q.  On rejection, for attempt = 1, 2, ...:
      y = philox(key, (i0, i1, attempt, 0)); the first accepted word of y0..y3.
  Gaussian (sigma = 3.2, |e| <= 19):
      x = philox(key, (i0 >> 1, i1, 0, 0)); h = i0 & 1
      magnitude = #{j in 0..18 : x[2h] >= T[j]},  negative iff magnitude > 0 and
      x[2h+1] is odd, with the cumulative table
      T[j] = floor(2^64 * P(|e| <= j)) of the discrete Gaussian
      rho(x) = exp(-x^2 / (2 sigma^2)) restricted to |x| <= 19.
"""
from __future__ import annotations

import decimal
from fractions import Fraction
from typing import List, Sequence

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B

QSEC, DBSEC, DBA, DBE, QA, QE = 1, 2, 3, 4, 5, 6
P_ID = 16            # stream id of the special prime

SIGMA_NUM, SIGMA_DEN = 32, 10     # sigma = 3.2, exactly
TAIL = 19

_U32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, m: int):
    """(hi, lo) 64-bit halves of the 128-bit product a * m, elementwise."""
    m0 = np.uint64(m & 0xFFFFFFFF)
    m1 = np.uint64(m >> 32)
    a0 = a & _U32
    a1 = a >> _S32
    p00 = a0 * m0
    p01 = a0 * m1
    p10 = a1 * m0
    p11 = a1 * m1
    mid = (p00 >> _S32) + (p01 & _U32) + (p10 & _U32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * np.uint64(m)
    return hi, lo


def philox4x64_10(k0: int, k1: int, c0, c1, c2, c3):
    """Philox4x64 with 10 rounds on arrays of counters; returns four uint64 arrays."""
    with np.errstate(over="ignore"):
        shape = np.broadcast(np.asarray(c0), np.asarray(c1), np.asarray(c2), np.asarray(c3)).shape
        x0 = np.broadcast_to(np.asarray(c0, dtype=np.uint64), shape).copy()
        x1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), shape).copy()
        x2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), shape).copy()
        x3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64), shape).copy()
        key0, key1 = k0 & (2**64 - 1), k1 & (2**64 - 1)
        for r in range(10):
            if r:
                key0 = (key0 + W0) & (2**64 - 1)
                key1 = (key1 + W1) & (2**64 - 1)
            hi0, lo0 = _mulhilo(x0, M0)
            hi1, lo1 = _mulhilo(x2, M1)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(key0), lo1,
                              hi0 ^ x3 ^ np.uint64(key1), lo0)
        return x0, x1, x2, x3


def tag(purpose: int, sub: int) -> int:
    return (purpose << 32) | sub


def uniform_mod(seed: int, purpose: int, sub: int, i0, i1, q: int) -> np.ndarray:
    """Uniform residues mod q (int64 array, q < 2^63) at element indices (i0, i1)."""
    i0 = np.asarray(i0, dtype=np.uint64)
    i1 = np.asarray(i1, dtype=np.uint64)
    i0, i1 = np.broadcast_arrays(i0, i1)
    key1 = tag(purpose, sub)
    bound = np.uint64(((1 << 64) // q) * q)
    blk = philox4x64_10(seed, key1, i0 >> np.uint64(2), i1, 0, 0)
    sel = (i0 & np.uint64(3)).astype(np.int64)
    w = np.choose(sel, blk)
    out = (w % np.uint64(q)).astype(np.int64)
    bad = np.nonzero(w >= bound)
    for idx in zip(*bad):            # rejection: astronomically rare for 36-bit q
        a0, a1 = int(i0[idx]), int(i1[idx])
        attempt = 1
        while True:
            y = philox4x64_10(seed, key1, a0, a1, attempt, 0)
            acc = [int(v) for v in y if int(v) < int(bound)]
            if acc:
                out[idx] = acc[0] % q
                break
            attempt += 1
    return out


def ternary(seed: int, purpose: int, sub: int, n: int) -> np.ndarray:
    """n ternary coefficients in {-1, 0, 1} (int64), uniform."""
    t = np.arange(n, dtype=np.uint64)
    return uniform_mod(seed, purpose, sub, t, np.zeros_like(t), 3) - 1


def _rho_decimal(x: int, prec: int) -> decimal.Decimal:
    ctx = decimal.Context(prec=prec)
    two_sigma2 = ctx.divide(decimal.Decimal(2 * SIGMA_NUM * SIGMA_NUM), decimal.Decimal(SIGMA_DEN * SIGMA_DEN))
    return ctx.exp(ctx.divide(decimal.Decimal(-x * x), two_sigma2))


def cdt_table(prec: int = 80) -> List[int]:
    """T[j] = floor(2^64 * P(|e| <= j)), j = 0..TAIL-1, truncated discrete Gaussian."""
    ctx = decimal.Context(prec=prec)
    rho = [_rho_decimal(x, prec) for x in range(TAIL + 1)]
    z = rho[0]
    for x in range(1, TAIL + 1):
        z = ctx.add(z, ctx.multiply(decimal.Decimal(2), rho[x]))
    out = []
    cum = rho[0]
    scale = decimal.Decimal(2) ** 64
    for j in range(TAIL):
        if j:
            cum = ctx.add(cum, ctx.multiply(decimal.Decimal(2), rho[j]))
        v = ctx.multiply(ctx.divide(cum, z), scale)
        out.append(int(v.to_integral_value(rounding=decimal.ROUND_FLOOR)))
    return out


_CDT = None


def _cdt() -> np.ndarray:
    global _CDT
    if _CDT is None:
        _CDT = np.array(cdt_table(), dtype=np.uint64)
    return _CDT


def _gauss_from_words(w: np.ndarray, sw: np.ndarray) -> np.ndarray:
    """Magnitude = #{j : w >= T[j]}; negative iff magnitude > 0 and sw is odd."""
    mag = np.searchsorted(_cdt(), w, side="right").astype(np.int64)
    neg = ((sw & np.uint64(1)) == np.uint64(1)) & (mag > 0)
    return np.where(neg, -mag, mag)


def gaussian(seed: int, purpose: int, sub: int, i0, i1) -> np.ndarray:
    """Discrete Gaussian integers (int64 array) at element indices (i0, i1)."""
    i0 = np.asarray(i0, dtype=np.uint64)
    i1 = np.asarray(i1, dtype=np.uint64)
    i0, i1 = np.broadcast_arrays(i0, i1)
    blk = philox4x64_10(seed, tag(purpose, sub), i0 >> np.uint64(1), i1, 0, 0)
    h = (i0 & np.uint64(1)).astype(bool)
    w = np.where(h, blk[2], blk[0])
    sw = np.where(h, blk[3], blk[1])
    return _gauss_from_words(w, sw)


def uniform_matrix(seed: int, purpose: int, sub: int, rows: int, cols: int, q: int) -> np.ndarray:
    """(rows x cols) int64 matrix; entry [r, c] is the uniform element (i0 = r, i1 = c).

    Same values as uniform_mod at those indices; each Philox block is computed
    once for the four consecutive rows it serves.
    """
    r4 = np.arange(-(-rows // 4), dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    blk = philox4x64_10(seed, tag(purpose, sub), r4, c, 0, 0)
    w = np.stack(blk, axis=1).reshape(-1, cols)[:rows]               # row 4*r4 + j <- word j
    bound = np.uint64(((1 << 64) // q) * q)
    out = (w % np.uint64(q)).astype(np.int64)
    bad = np.nonzero(w >= bound)
    if bad[0].size:
        out[bad] = uniform_mod(seed, purpose, sub, bad[0].astype(np.uint64),
                               bad[1].astype(np.uint64), q)
    return out


def uniform_columns(seed: int, purpose: int, sub: int, rows: int, c0: int, c1: int, q: int) -> np.ndarray:
    """(rows x (c1 - c0)) int64 matrix whose column j is elements (i0 = 0..rows-1, i1 = c0 + j): the
    same values as uniform_matrix, for large sizes.

    For a fixed column i1 the counters (i0 >> 2, i1, 0, 0) run through consecutive values of word 0,
    so one column is the raw output of numpy's Philox4x64-10 bit generator (an independent library
    implementation of the same published generator) started at that column's first counter.  numpy
    increments its 256-bit counter before each block, so the generator is seeded one below it.
    Words w >= floor(2^64 / q) q take the rejection path of uniform_mod.
    """
    blocks = -(-rows // 4)
    out = np.empty((rows, c1 - c0), dtype=np.int64)
    bound = np.uint64(((1 << 64) // q) * q)
    key = np.array([seed & (2**64 - 1), tag(purpose, sub)], dtype=np.uint64)
    for j, c in enumerate(range(c0, c1)):
        ctr = (c << 64) - 1 if c else (1 << 256) - 1            # 256-bit counter (0, c, 0, 0) minus one
        words = [(ctr >> (64 * t)) & (2**64 - 1) for t in range(4)]
        g = np.random.Philox(key=key, counter=np.array(words, dtype=np.uint64))
        w = g.random_raw(4 * blocks)[:rows]
        col = (w % np.uint64(q)).astype(np.int64)
        bad = np.nonzero(w >= bound)[0]
        if bad.size:
            col[bad] = uniform_mod(seed, purpose, sub, bad.astype(np.uint64),
                                   np.full(bad.size, c, dtype=np.uint64), q)
        out[:, j] = col
    return out


def gaussian_matrix(seed: int, purpose: int, sub: int, rows: int, cols: int) -> np.ndarray:
    """(rows x cols) Gaussian integers; entry [r, c] is element (i0 = r, i1 = c)."""
    r2 = np.arange(-(-rows // 2), dtype=np.uint64)[:, None]
    c = np.arange(cols, dtype=np.uint64)[None, :]
    x0, x1, x2, x3 = philox4x64_10(seed, tag(purpose, sub), r2, c, 0, 0)
    w = np.stack([x0, x2], axis=1).reshape(-1, cols)[:rows]
    sw = np.stack([x1, x3], axis=1).reshape(-1, cols)[:rows]
    return _gauss_from_words(w, sw)


def gaussian_pmf() -> List[Fraction]:
    """P(|e| = j), j = 0..TAIL, as exact fractions of the sampler's table."""
    T = [0] + cdt_table() + [1 << 64]
    return [Fraction(T[j + 1] - T[j], 1 << 64) for j in range(TAIL + 1)]
