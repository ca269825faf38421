"""Negacyclic ring products and exact integer matrix products (oracle).

Ring R_n = Z[X]/(X^n + 1) (Section 2.2.1): X^n = -1, so a coefficient that
wraps past degree n - 1 changes sign.  For s in R_n the n x n matrix
Neg(s)[t][v] = s[t - v] if t >= v else -s[t - v + n]
satisfies coeffs(s * a) = Neg(s) @ coeffs(a), which is the schoolbook product
written as a matrix; stacking Neg(s_j) of several secrets gives the secret
matrices S_Q and S_DB of the CCMM.

All products here are exact integer arithmetic.  `imatmul` runs torch int64
matrix products on the CPU and asserts beforehand that no partial sum can
exceed 2^62 in magnitude; `modmatmul` splits 36-bit residues into 18-bit limbs
so that every limb product sum fits that bound, then recombines the limbs with
Python integers.
"""
from __future__ import annotations

from typing import List

import numpy as np
import torch

_LIMIT = 1 << 62


def neg_matrix(s: np.ndarray, rows: int | None = None) -> np.ndarray:
    """Neg(s) restricted to its first `rows` rows (int64)."""
    n = len(s)
    rows = n if rows is None else rows
    t = np.arange(rows)[:, None]
    v = np.arange(n)[None, :]
    d = t - v
    out = np.where(d >= 0, s[d % n], -s[d % n])
    return out.astype(np.int64)


def negmul_schoolbook(s, a) -> List[int]:
    """Schoolbook product s * a in Z[X]/(X^n + 1) with Python integers (tiny n only)."""
    n = len(s)
    out = [0] * n
    for u in range(n):
        for v in range(n):
            if s[u] == 0 or a[v] == 0:
                continue
            w = u + v
            if w < n:
                out[w] += int(s[u]) * int(a[v])
            else:
                out[w - n] -= int(s[u]) * int(a[v])
    return out


def _maxabs(x: np.ndarray) -> int:
    if x.size == 0:
        return 0
    return int(max(abs(int(x.max())), abs(int(x.min()))))


def imatmul(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Exact A @ B for int64 matrices whose partial sums stay below 2^62."""
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    K = A.shape[-1]
    assert B.shape[0] == K
    bound = _maxabs(A) * _maxabs(B) * max(K, 1)
    assert bound < _LIMIT, "imatmul: partial sums could overflow int64"
    if A.size == 0 or B.size == 0:
        return np.zeros((A.shape[0], B.shape[1]), dtype=np.int64)
    if A.shape[0] * B.shape[1] * K < (1 << 22):
        return A @ B                 # small products: numpy's int64 loop has less overhead
    return torch.from_numpy(np.ascontiguousarray(A)).matmul(
        torch.from_numpy(np.ascontiguousarray(B))).numpy()


def modmatmul(A: np.ndarray, B: np.ndarray, q: int) -> np.ndarray:
    """(A @ B) mod q for residue matrices with entries in [0, 2^36); int64 result in [0, q)."""
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    assert A.min(initial=0) >= 0 and B.min(initial=0) >= 0
    assert A.max(initial=0) < (1 << 36) and B.max(initial=0) < (1 << 36)
    m = (1 << 18) - 1
    a0, a1 = A & m, A >> 18
    b0, b1 = B & m, B >> 18
    p00 = imatmul(a0, b0)
    p01 = imatmul(a0, b1)
    p10 = imatmul(a1, b0)
    p11 = imatmul(a1, b1)
    out = np.empty(p00.shape, dtype=np.int64)
    for idx in np.ndindex(out.shape):
        v = (int(p11[idx]) << 36) + ((int(p01[idx]) + int(p10[idx])) << 18) + int(p00[idx])
        out[idx] = v % q
    return out
