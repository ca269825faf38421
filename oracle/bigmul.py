"""Exact negacyclic products for large ring degrees (oracle).

Products in Z_q[X]/(X^n + 1) of two arbitrary residue polynomials at n up to 2^16, where the
Neg(s)-matrix form of ring.py would need n^2 entries.  Each operand is cut into 12-bit limbs; every
limb product is a linear convolution computed with numpy's real FFT of length 2n and rounded to the
nearest integer, which is exact because the true coefficients are integers below n 2^24 <= 2^40 and
the FFT's error at that size stays far below 1/2 (asserted on every call: the largest distance of the
FFT output from an integer must stay below 1/16).  The limb products are folded by X^n = -1 and
recombined mod q with Python integers.  The FFT serves only as the library primitive that multiplies
polynomials; everything around it is the definition (s * a)_t = sum_u s_u a_{t-u}, negated on wrap.
"""
from __future__ import annotations

import numpy as np

LIMB = 12


def _limbs(a: np.ndarray, bits: int):
    """Non-negative int64 a (< 2^bits) -> list of 12-bit limb arrays, least significant first."""
    out = []
    x = a.copy()
    for _ in range(-(-bits // LIMB)):
        out.append((x & ((1 << LIMB) - 1)).astype(np.float64))
        x >>= LIMB
    return out


def _conv(x: np.ndarray, y: np.ndarray, n: int) -> np.ndarray:
    """Exact linear convolution (length 2n) of two non-negative limb arrays, as int64."""
    fx = np.fft.rfft(x, 2 * n)
    fy = np.fft.rfft(y, 2 * n)
    z = np.fft.irfft(fx * fy, 2 * n)
    r = np.rint(z)
    assert float(np.max(np.abs(z - r))) < 1.0 / 16, "FFT rounding too close to 1/2: product not exact"
    return r.astype(np.int64)


def negmul_mod(s: np.ndarray, a: np.ndarray, q: int) -> np.ndarray:
    """(s * a) mod (X^n + 1, q) for residue polynomials s, a (entries in [0, q), q < 2^62), as int64."""
    s = np.asarray(s, dtype=np.int64) % q
    a = np.asarray(a, dtype=np.int64) % q
    n = len(s)
    assert len(a) == n
    bits = max(int(q - 1).bit_length(), 1)
    ls, la = _limbs(s, bits), _limbs(a, bits)
    acc = np.zeros(n, dtype=object)
    for i, x in enumerate(ls):
        for j, y in enumerate(la):
            c = _conv(x, y, n)
            folded = c[:n] - c[n:]                       # X^n = -1
            acc = acc + folded.astype(object) * (1 << (LIMB * (i + j)))
    return np.array([int(v) % q for v in acc], dtype=np.int64)


def negmul_small(s: np.ndarray, a: np.ndarray, q: int) -> np.ndarray:
    """(s * a) mod (X^n + 1, q) for a small signed s (|s_u| <= 1, e.g. a ternary secret) and residues a."""
    s = np.asarray(s, dtype=np.int64)
    assert int(np.max(np.abs(s))) <= 1
    return negmul_mod(s % q, a, q)
