"""The CCMM over the paper's own modulus chain: moduli n^2 for primes 127 <= n <= 253 (oracle).

Section 6.3 ("Fast PPMM using int8 cuBLAS") takes the ciphertext modulus itself as a product of
squares of small primes, Q = prod n^2 over the primes 127 <= n <= 253, so that a product modulo Q is a
product modulo each n^2, and each of those is three int8 products of the digits M + n M'.  This
module is the same scheme as oracle/ckks.py (Section 2.3: shared-a query ciphertexts, the RGSW-style
database pair, the four plaintext products written as one product per modulus, the rescale of
Section 2.2.4, decryption of Section 2.2.2) with that modulus family in place of the 36-bit NTT primes:

  query modulus       Q_l = m_0 ... m_{l-1}            (m_j = n_j^2, the first l query bases)
  special part        P   = m'_0 ... m'_{r-1}          (the next r bases; P plays the role of p)
  database modulus    Q_L P
  database scale      P:   B = -S_DB A + P [M_DB | T] + E  (mod each modulus)
  query scale         Delta_l = 2^(floor(log2 Q_l) - gap)
  CCMM                C = D X mod each modulus of Q_l P, X the centered lift of the query from Q_l;
                      result RS_P(C) = floor(C / P + 1/2) mod Q_l   (P odd: no ties)

Readings (the paper is silent on them): the query bases are the largest primes of the range first,
the special part the next ones; random draws per modulus use the stream id 256 + n (a residue mod n^2
is uniform, independently per modulus, which is uniform mod the product by the CRT); the error
integers and the secrets are those of the prime family (the same streams), so one integer error e
is added under every modulus.

Residue arrays are int64 with entries in [0, n^2).  Every function keeps to the plain definition
(Python integers for CRT and rescale, exact int64 matrix products) and shares no code with the GPU
library, which never calls into this module.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import prng
from .ckks import Keys, centered, crt, keygen, s_db_rows, s_q_matrix
from .params import Params, is_prime
from .ring import imatmul, modmatmul

# the primes n with 127 <= n <= 253, largest first (Section 6.3: 24 of them, 48 int8 planes)
CHAIN_BASES: Tuple[int, ...] = tuple(n for n in range(253, 126, -1) if is_prime(n))


def stream_id(n: int) -> int:
    """Random-stream id of the modulus n^2."""
    return 256 + n


@dataclasses.dataclass(frozen=True)
class ChainParams:
    log_n_db: int
    log_n_q: int
    q_bases: Tuple[int, ...]     # n_0 .. n_{L-1}: query moduli n_j^2
    p_bases: Tuple[int, ...]     # the special part's bases
    d2: int
    max_db_rows: int
    gap: int = 20
    t_num: int = 3
    t_den: int = 8

    @property
    def ring(self) -> Params:
        """The ring shapes (for the secrets, which the chain shares with the prime family)."""
        return Params(log_n_db=self.log_n_db, log_n_q=self.log_n_q, q=(), p=0, d2=self.d2,
                      max_db_rows=self.max_db_rows, gap=self.gap)

    @property
    def n_db(self) -> int:
        return 1 << self.log_n_db

    @property
    def n_q(self) -> int:
        return 1 << self.log_n_q

    @property
    def K(self) -> int:
        return self.d2 + self.n_q

    def q_mods(self, level: int) -> List[int]:
        return [n * n for n in self.q_bases[:level]]

    @property
    def p_mods(self) -> List[int]:
        return [n * n for n in self.p_bases]

    def Q(self, level: int) -> int:
        out = 1
        for m in self.q_mods(level):
            out *= m
        return out

    @property
    def P(self) -> int:
        out = 1
        for m in self.p_mods:
            out *= m
        return out

    def delta(self, level: int) -> int:
        return 1 << (self.Q(level).bit_length() - 1 - self.gap)

    def all_bases(self) -> List[int]:
        """Database modulus order: the query bases, then the special part's."""
        return list(self.q_bases) + list(self.p_bases)


def make_chain_params(log_n_db: int, log_n_q: int, n_q_mods: int, n_p_mods: int, d2: int,
                      max_db_rows: int, gap: int = 20) -> ChainParams:
    """The largest n_q_mods primes of the range for Q, the next n_p_mods for P."""
    assert n_q_mods + n_p_mods <= len(CHAIN_BASES)
    return ChainParams(log_n_db=log_n_db, log_n_q=log_n_q, q_bases=CHAIN_BASES[:n_q_mods],
                       p_bases=CHAIN_BASES[n_q_mods:n_q_mods + n_p_mods], d2=d2, max_db_rows=max_db_rows,
                       gap=gap)


def chain_keygen(C: ChainParams, seed: int) -> Keys:
    """The ternary secrets (the prime family's streams): s_j in R_{N_Q}, s'_j in R_{N_DB}."""
    return keygen(C.ring, seed)


# ---------------------------------------------------------------- encryption

def encrypt_db(C: ChainParams, keys: Keys, m_db: np.ndarray, seed: int) -> Dict[int, np.ndarray]:
    """D per base n (modulus n^2), for every query base and the special part's:
    (N_DB + d1) x (d2 + N_Q) with D = [[A], [B]], B = -S_DB A + P [M_DB | T] + E (mod n^2)."""
    d1, d2 = m_db.shape
    assert d2 == C.d2 and d1 <= C.max_db_rows
    SQ = s_q_matrix(keys)
    SDB = s_db_rows(keys, range(d1))
    T = imatmul(m_db.astype(np.int64), SQ)                               # d1 x N_Q, exact
    plain = np.concatenate([m_db.astype(np.int64), T], axis=1)           # [M_DB | T]
    E = prng.gaussian_matrix(seed, prng.DBE, 0, d1, C.K)
    out = {}
    for n in C.all_bases():
        m = n * n
        A = prng.uniform_matrix(seed, prng.DBA, stream_id(n), C.n_db, C.K, m)
        B = (-imatmul(SDB, A) + (C.P % m) * plain + E) % m
        out[n] = np.concatenate([A, B], axis=0)
    return out


def encrypt_query(C: ChainParams, keys: Keys, m_q_rows: np.ndarray, level: int, seed: int) -> Dict[int, np.ndarray]:
    """XT per query base n < level: d3 x (d2 + N_Q), row c = [b_c | a_c] with
    b_c = -S_Q a_c + Delta_level m_c + e_c (mod n^2)."""
    d3, d2 = m_q_rows.shape
    assert d2 == C.d2 and 1 <= level <= len(C.q_bases)
    SQ = s_q_matrix(keys)
    MQ = m_q_rows.astype(np.int64).T                                      # d2 x d3
    E = prng.gaussian_matrix(seed, prng.QE, 0, d2, d3)
    delta = C.delta(level)
    out = {}
    for n in C.q_bases[:level]:
        m = n * n
        A = prng.uniform_matrix(seed, prng.QA, stream_id(n), C.n_q, d3, m)
        B = (-imatmul(SQ, A) + (delta % m) * MQ + E) % m
        out[n] = np.concatenate([B.T, A.T], axis=1)
    return out


# ---------------------------------------------------------------- CCMM

def lift_query(C: ChainParams, XT: Dict[int, np.ndarray], level: int) -> List[List[int]]:
    """L(x): the centered representative mod Q_level of every query residue vector."""
    bases = C.q_bases[:level]
    moduli = [n * n for n in bases]
    Q = C.Q(level)
    d3, K = XT[bases[0]].shape
    return [[centered(crt([int(XT[n][c, k]) for n in bases], moduli), Q) for k in range(K)] for c in range(d3)]


def ccmm_pre_rescale(C: ChainParams, D: Dict[int, np.ndarray], XT: Dict[int, np.ndarray], level: int,
                     row0: int, rows: int) -> Dict[int, np.ndarray]:
    """C = D_sel X mod n^2 for the level's query bases and the special part's: (N_DB + rows) x d3."""
    L = lift_query(C, XT, level)
    sel = np.concatenate([np.arange(C.n_db), C.n_db + row0 + np.arange(rows)])
    out = {}
    for n in list(C.q_bases[:level]) + list(C.p_bases):
        m = n * n
        X = np.array([[v % m for v in col] for col in L], dtype=np.int64).T    # K x d3
        out[n] = modmatmul(D[n][sel], X, m)
    return out


def rescale(x: int, P: int, Q: int) -> int:
    """RS_P(x) = floor(x / P + 1/2) mod Q for an integer x (P odd: no ties)."""
    return ((2 * x + P) // (2 * P)) % Q


def ccmm(C: ChainParams, D: Dict[int, np.ndarray], XT: Dict[int, np.ndarray], level: int,
         row0: int, rows: int) -> Dict[int, np.ndarray]:
    """Result per query base n < level: d3 x (N_DB + rows), [A_out | B_out] per column (mod n^2)."""
    pre = ccmm_pre_rescale(C, D, XT, level, row0, rows)
    bases = list(C.q_bases[:level]) + list(C.p_bases)
    moduli = [n * n for n in bases]
    Q, P = C.Q(level), C.P
    R, d3 = pre[bases[0]].shape
    res = {n: np.empty((d3, R), dtype=np.int64) for n in C.q_bases[:level]}
    for r in range(R):
        for c in range(d3):
            x = crt([int(pre[n][r, c]) for n in bases], moduli)       # in [0, Q P)
            y = rescale(x, P, Q)
            for n in C.q_bases[:level]:
                res[n][c, r] = y % (n * n)
    return res


# ---------------------------------------------------------------- decryption

def decrypt(C: ChainParams, keys: Keys, out: Dict[int, np.ndarray], level: int, row0: int, rows: int
            ) -> Tuple[List[List[Fraction]], np.ndarray]:
    """(v, IP): v = centered(B_out + S_DB A_out mod Q_level) / Delta; IP = floor(v + 1/2)."""
    bases = C.q_bases[:level]
    moduli = [n * n for n in bases]
    Q = C.Q(level)
    delta = C.delta(level)
    S = s_db_rows(keys, range(row0, row0 + rows))
    y = {}
    for n in bases:
        A_out = out[n][:, :C.n_db]
        B_out = out[n][:, C.n_db:]
        y[n] = (B_out + imatmul(A_out, S.T)) % (n * n)
    d3 = out[bases[0]].shape[0]
    v = [[Fraction(0)] * rows for _ in range(d3)]
    ip = np.empty((d3, rows), dtype=np.int64)
    for c in range(d3):
        for r in range(rows):
            yc = centered(crt([int(y[n][c, r]) for n in bases], moduli), Q)
            v[c][r] = Fraction(yc, delta)
            ip[c, r] = (2 * yc + delta) // (2 * delta)
    return v, ip
