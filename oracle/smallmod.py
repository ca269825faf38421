"""Small-modulus int8 forms of a modular matrix product (Section 6.3, fast plaintext matrix
products with int8 arithmetic).  Test infrastructure, like the rest of the oracle.

The paper reduces a matrix product modulo a large modulus to int8 matrix products by two
techniques:

* RNS over small pairwise coprime moduli (each below 2^8): the product modulo each small modulus
  is one int8 matrix product;
* the split of a matrix modulo n^2 as M + n M' (|entries| < n): the product modulo n^2 follows
  from MN + n (M'N + MN') (mod n^2), i.e. three int8 matrix products.

Here they serve the product of matrices whose entries are residues modulo a 36-bit prime q: the
entries are taken as centered integers, the exact integer product S is recovered from its
residues modulo small moduli whose product exceeds 2 max|S| (Chinese remaindering), and S is
reduced modulo q.  This gives the same C = A B mod q as the digit form, by another route.

Plain Python integers and numpy int64; products of int8 planes use the exact integer matmul of
oracle.ring.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from .ring import imatmul

# Pairwise coprime moduli <= 256 (balanced residues fit int8), largest product first:
# 2^8, 3*5*17, 11*23, 251, 13*19, then primes.
RNS_MODULI: Tuple[int, ...] = (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191)


def _is_prime(n: int) -> bool:
    return n > 1 and all(n % d for d in range(2, math.isqrt(n) + 1))


# Bases n of the n^2 split: the primes 127 <= n <= 253 of the paper's modulus, largest first.
P2_BASES: Tuple[int, ...] = tuple(sorted((p for p in range(127, 254) if _is_prime(p)), reverse=True))


def centered(x, q: int):
    """Representative of x mod q in (-q/2, q/2] (numpy int64 arrays or Python ints)."""
    r = np.mod(x, q) if isinstance(x, np.ndarray) else x % q
    return np.where(r > q // 2, r - q, r) if isinstance(r, np.ndarray) else (r - q if r > q // 2 else r)


def balanced(x, m: int):
    """Representative of x mod m in [-floor(m/2), ceil(m/2) - 1]: fits int8 for m <= 256."""
    r = np.mod(x, m)
    return np.where(r >= (m + 1) // 2, r - m, r)


def product_bound(K: int, q: int) -> int:
    """2 max|S| + 1 for S = sum of K products of centered residues mod q."""
    h = (q - 1) // 2
    return 2 * K * h * h + 1


def rns_moduli_for(K: int, q: int) -> Tuple[int, ...]:
    """The shortest prefix of RNS_MODULI whose product covers product_bound(K, q)."""
    prod, out = 1, []
    for m in RNS_MODULI:
        out.append(m)
        prod *= m
        if prod >= product_bound(K, q):
            return tuple(out)
    raise ValueError("K too large for the RNS moduli")


def p2_bases_for(K: int, q: int) -> Tuple[int, ...]:
    """The shortest prefix of P2_BASES whose squares' product covers product_bound(K, q)."""
    prod, out = 1, []
    for n in P2_BASES:
        out.append(n)
        prod *= n * n
        if prod >= product_bound(K, q):
            return tuple(out)
    raise ValueError("K too large for the n^2 bases")


def crt(residues: Sequence[int], moduli: Sequence[int]) -> int:
    """The integer in [0, prod moduli) with the given residues (pairwise coprime moduli)."""
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def rns_split(Xc: np.ndarray, moduli: Sequence[int]) -> List[np.ndarray]:
    """One int8 plane per modulus: the balanced residue of each centered entry."""
    return [balanced(Xc, m).astype(np.int8) for m in moduli]


def p2_split(Xc: np.ndarray, n: int) -> Tuple[np.ndarray, np.ndarray]:
    """(M, M') with Xc = M + n M' (mod n^2), both balanced mod n (int8)."""
    r = np.mod(Xc, n * n)
    M = balanced(r, n)
    Mp = balanced((r - M) // n, n)
    return M.astype(np.int8), Mp.astype(np.int8)


def _reduce_mod_q(res_per_mod: List[np.ndarray], moduli: Sequence[int], q: int) -> np.ndarray:
    """Entrywise CRT of the residue matrices to the centered exact integer, then mod q."""
    M = 1
    for m in moduli:
        M *= m
    shape = res_per_mod[0].shape
    out = np.empty(shape, dtype=np.int64)
    flat = [r.reshape(-1) for r in res_per_mod]
    o = out.reshape(-1)
    for i in range(o.size):
        x = crt([int(f[i]) for f in flat], moduli)
        if x > M // 2:
            x -= M
        o[i] = x % q
    return out


def rns_matmul_mod(A: np.ndarray, B: np.ndarray, q: int, moduli: Sequence[int] = None) -> np.ndarray:
    """C = A B mod q via one int8 product per small modulus (RNS technique)."""
    Ac, Bc = centered(A.astype(np.int64), q), centered(B.astype(np.int64), q)
    moduli = moduli or rns_moduli_for(A.shape[1], q)
    res = []
    for m, Am, Bm in zip(moduli, rns_split(Ac, moduli), rns_split(Bc, moduli)):
        res.append(np.mod(imatmul(Am.astype(np.int64), Bm.astype(np.int64)), m))
    return _reduce_mod_q(res, moduli, q)


def p2_matmul_mod(A: np.ndarray, B: np.ndarray, q: int, bases: Sequence[int] = None) -> np.ndarray:
    """C = A B mod q via three int8 products per modulus n^2 (the M + n M' technique)."""
    Ac, Bc = centered(A.astype(np.int64), q), centered(B.astype(np.int64), q)
    bases = bases or p2_bases_for(A.shape[1], q)
    res = []
    for n in bases:
        M, Mp = p2_split(Ac, n)
        N, Np = p2_split(Bc, n)
        M, Mp, N, Np = (x.astype(np.int64) for x in (M, Mp, N, Np))
        G0 = imatmul(M, N)
        G1 = imatmul(M, Np) + imatmul(Mp, N)
        res.append(np.mod(G0 + n * G1, n * n))
    return _reduce_mod_q(res, [n * n for n in bases], q)
