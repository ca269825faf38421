"""FormatSwitch: the query from its transmission ring to the CCMM's MSRLWE format (oracle).

Appendix C.1 of the paper (query preprocessing, "FormatSwitch" of Table 3): the query arrives as RLWE
ciphertexts of ring degree N_T = 2^16; each is ring-switched to degree N_Q = 2^13 by key switching to
a secret of R_{N_Q} embedded as s'(X^(N_T/N_Q)) and taking the trace, which on the key-switched
ciphertext is the extraction of the coefficients of degree divisible by rho = N_T / N_Q; each pair of
half codes is converted to the MSRLWE (shared-a) format; and the scale is brought to the CCMM's by a
modulus switch.  This module writes those steps out in coefficient encoding, the encoding the CCMM
consumes:

  transmission   chunk j of query column c (code positions [j N_Q, (j+1) N_Q) of the d2) at the
                 coefficients rho u of an RLWE ciphertext (a, b) in R_{N_T} mod Q' = q_0 .. q_l under
                 s_T:  b = -a s_T + (Delta_l q_l) m~ + e
  key switching  digits d_i = [a (Q'/q_i)^-1]_{q_i} (i <= l, one per prime), keys
                 K_i = (k_i, -k_i s_to + p (Q'/q_i) s_from + e_i) mod Q' p;  KS(a) = RS_p(sum_i d_i K_i)
                 (RS_p(x) = floor(x / p + 1/2) mod Q', Section 2.2.4), so that B + A s_to ~ a s_from
  ring switch    (A, b + B) := KS_{s_T -> s'(X^rho)}(a);  a'(Y) = sum_u A_{rho u} Y^u,  b' likewise
  conversion     the k chunks (a'_j, b'_j) under s' to (a, b_0 .. b_{k-1}) under the CCMM secrets
                 s_0 .. s_{k-1}: keys K_{i,j,j'} = (k_{i,j}, -k_{i,j} s_j' + [j = j'] p (Q'/q_i) s' + e)
                 with k_{i,j} shared by the outputs j', a = RS_p(sum_{i,j} d_i(a'_j) k_{i,j}),
                 b_j' = b'_j' + RS_p(sum_{i,j} d_i(a'_j) (-k_{i,j} s_j' + ...))
  modulus switch RS_{q_l} from Q' to Q_l = q_0 .. q_{l-1}: scale Delta_l q_l -> Delta_l

Readings (the paper leaves them open; listed in the design notes): coefficient encoding with the
chunks placed at degrees divisible by rho (the slot-domain masking that isolates a half code before
the trace is then not needed: each half code is its own transmission ciphertext); one digit per prime
(the paper's dnum 8 over 8 primes); the special prime p of the CCMM keys as the key-switching modulus;
the conversion keys above (one random polynomial per digit and input chunk, shared by the k outputs,
which is what makes the output's a common); random streams of new purposes (below); non-negative
digits.  Products in R_{N_T} use oracle.bigmul (exact through an FFT with an integrality check).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np

from . import prng
from .bigmul import negmul_mod
from .ckks import Keys, centered, keygen
from .params import Params

TSEC, RSEC, RKA, RKE, CKA, CKE, TA, TE = 7, 8, 9, 10, 11, 12, 13, 14


@dataclasses.dataclass
class FSKeys:
    P: Params
    level: int                    # CCMM level l: transmission at l + 1 primes
    log_n_t: int
    keys: Keys                    # the CCMM keys (secrets s_j of the query layer)
    s_t: np.ndarray               # transmission secret, N_T ternary
    s_r: np.ndarray               # ring-switch secret s', N_Q ternary
    rk: Dict[int, List[Tuple[np.ndarray, np.ndarray]]]      # prime -> [(k_i, beta_i)], i <= l
    ck: Dict[int, List[List[Tuple[np.ndarray, List[np.ndarray]]]]]   # prime -> [i][j] (k_ij, [beta_ij j'])

    @property
    def n_t(self) -> int:
        return 1 << self.log_n_t

    @property
    def rho(self) -> int:
        return self.n_t // self.P.n_q

    def primes_in(self) -> List[int]:
        """Q' = q_0 .. q_l."""
        return [self.P.q[i] for i in range(self.level + 1)]

    def ids(self) -> List[Tuple[int, int]]:
        """(stream id, prime) of Q' and p."""
        return [(i, self.P.q[i]) for i in range(self.level + 1)] + [(prng.P_ID, self.P.p)]


def _ternary(seed, purpose, n):
    return prng.ternary(seed, purpose, 0, n)


def _embed(s: np.ndarray, rho: int) -> np.ndarray:
    """s(X^rho) in R_{rho n}."""
    out = np.zeros(len(s) * rho, dtype=np.int64)
    out[::rho] = s
    return out


def fs_keygen(P: Params, level: int, log_n_t: int, seed: int) -> FSKeys:
    """CCMM keys (ckks.keygen) plus s_T, s' and the ring-switch and conversion keys for level `level`."""
    assert 1 <= level and level + 1 <= len(P.q)
    keys = keygen(P, seed)
    n_t, n_q = 1 << log_n_t, P.n_q
    rho = n_t // n_q
    assert rho * n_q == n_t and rho >= 1
    s_t = _ternary(seed, TSEC, n_t)
    s_r = _ternary(seed, RSEC, n_q)
    s_emb = _embed(s_r, rho)
    primes = [P.q[i] for i in range(level + 1)]
    Qp = 1
    for q in primes:
        Qp *= q
    ids = [(i, P.q[i]) for i in range(level + 1)] + [(prng.P_ID, P.p)]
    k = P.k
    t_n, t_q = np.arange(n_t, dtype=np.uint64), np.arange(n_q, dtype=np.uint64)
    rk, ck = {}, {}
    for pid, z in ids:
        rk[z] = []
        for i, qi in enumerate(primes):
            gi = (P.p * (Qp // qi)) % z
            ka = prng.uniform_mod(seed, RKA, pid, t_n, np.full(n_t, i, dtype=np.uint64), z)
            e = prng.gaussian(seed, RKE, 0, t_n, np.full(n_t, i, dtype=np.uint64))
            beta = (-negmul_mod(s_emb % z, ka, z) + gi * s_t + e) % z          # |gi s_T| < 2^36
            rk[z].append((ka, beta))
        ck[z] = []
        for i, qi in enumerate(primes):
            gi = (P.p * (Qp // qi)) % z
            row = []
            for j in range(k):
                idx = i * k + j
                ka = prng.uniform_mod(seed, CKA, pid, t_q, np.full(n_q, idx, dtype=np.uint64), z)
                betas = []
                for jp in range(k):
                    e = prng.gaussian(seed, CKE, 0, t_q, np.full(n_q, idx * k + jp, dtype=np.uint64))
                    b = -negmul_mod(keys.s[jp] % z, ka, z) + e
                    if j == jp:
                        b = b + gi * s_r                                              # |gi s'| < 2^36
                    betas.append(b % z)
                row.append((ka, betas))
            ck[z].append(row)
    return FSKeys(P, level, log_n_t, keys, s_t, s_r, rk, ck)


def encrypt_transmit(F: FSKeys, m_q_rows: np.ndarray, seed: int) -> Dict[int, np.ndarray]:
    """Transmission ciphertexts per prime of Q': [d3 k][2][N_T] = (a, b) of column c, chunk j at c k + j,
    b = -a s_T + (Delta_l q_l) m~ + e with m~_{rho u} = m[c][j N_Q + u]."""
    P, lvl = F.P, F.level
    d3, d2 = m_q_rows.shape
    assert d2 == P.d2
    n_t, n_q, rho, k = F.n_t, P.n_q, F.rho, P.k
    scale = P.delta(lvl) * P.q[lvl]
    t_n = np.arange(n_t, dtype=np.uint64)
    out = {q: np.zeros((d3 * k, 2, n_t), dtype=np.int64) for q in F.primes_in()}
    for c in range(d3):
        for j in range(k):
            col = c * k + j
            mt = np.zeros(n_t, dtype=np.int64)
            lo, hi = j * n_q, min((j + 1) * n_q, d2)
            mt[: (hi - lo) * rho: rho] = m_q_rows[c, lo:hi]
            e = prng.gaussian(seed, TE, 0, t_n, np.full(n_t, col, dtype=np.uint64))
            for i, q in enumerate(F.primes_in()):
                a = prng.uniform_mod(seed, TA, i, t_n, np.full(n_t, col, dtype=np.uint64), q)
                b = (-negmul_mod(F.s_t % q, a, q) + (scale % q) * mt + e) % q
                out[q][col, 0] = a
                out[q][col, 1] = b
    return out


def digits(a_res: Dict[int, np.ndarray], primes: List[int]) -> List[np.ndarray]:
    """d_i = [a (Q'/q_i)^-1]_{q_i} in [0, q_i), one integer polynomial per prime of Q'."""
    Qp = 1
    for q in primes:
        Qp *= q
    return [np.array([int(x) * pow((Qp // q) % q, -1, q) % q for x in a_res[q]], dtype=np.int64) for q in primes]


def rescale_by(res: Dict[int, np.ndarray], div: int, keep: List[int]) -> Dict[int, np.ndarray]:
    """RS_div: x (residues over keep + [div]) -> floor(x / div + 1/2) mod prod(keep), per prime of keep:
    (x_z - [x_div]_centered) div^-1 mod z."""
    xc = np.array([centered(int(v), div) for v in res[div]], dtype=object)
    out = {}
    for z in keep:
        inv = pow(div % z, -1, z)
        out[z] = np.array([(int(x) - int(c)) * inv % z for x, c in zip(res[z], xc)], dtype=np.int64)
    return out


def key_switch(F: FSKeys, a_res: Dict[int, np.ndarray], key_of) -> Tuple[Dict[int, np.ndarray], Dict]:
    """sum_i d_i(a) K_i, rescaled by p: key_of(z, i) -> (k, beta) residues mod z."""
    primes = F.primes_in()
    d = digits(a_res, primes)
    A, B = {}, {}
    for pid, z in F.ids():
        acc_a = np.zeros(len(a_res[primes[0]]), dtype=np.int64)
        acc_b = np.zeros_like(acc_a)
        for i in range(len(primes)):
            ka, beta = key_of(z, i)
            acc_a = (acc_a + negmul_mod(d[i] % z, ka, z)) % z
            acc_b = (acc_b + negmul_mod(d[i] % z, beta, z)) % z
        A[z], B[z] = acc_a, acc_b
    return rescale_by(A, F.P.p, primes), rescale_by(B, F.P.p, primes)


def ring_switch(F: FSKeys, ct: Dict[int, np.ndarray], col: int):
    """Transmission ciphertext `col` -> (a', b') in R_{N_Q} mod Q' under s'."""
    primes = F.primes_in()
    a = {q: ct[q][col, 0] for q in primes}
    b = {q: ct[q][col, 1] for q in primes}
    A, B = key_switch(F, a, lambda z, i: F.rk[z][i])
    rho = F.rho
    return ({q: A[q][::rho].copy() for q in primes}, {q: ((b[q] + B[q]) % q)[::rho].copy() for q in primes})


def convert(F: FSKeys, chunks) -> Tuple[Dict[int, np.ndarray], List[Dict[int, np.ndarray]]]:
    """k RLWE ciphertexts (a'_j, b'_j) under s' -> MSRLWE (a, b_0 .. b_{k-1}) under s_0 .. s_{k-1}."""
    primes = F.primes_in()
    k = F.P.k
    dig = [digits(a_j, primes) for a_j, _ in chunks]
    n_q = F.P.n_q
    A = {}
    Bs = [dict() for _ in range(k)]
    for pid, z in F.ids():
        acc_a = np.zeros(n_q, dtype=np.int64)
        acc_b = [np.zeros(n_q, dtype=np.int64) for _ in range(k)]
        for i in range(len(primes)):
            for j in range(k):
                ka, betas = F.ck[z][i][j]
                dz = dig[j][i] % z
                acc_a = (acc_a + negmul_mod(dz, ka, z)) % z
                for jp in range(k):
                    acc_b[jp] = (acc_b[jp] + negmul_mod(dz, betas[jp], z)) % z
        A[z] = acc_a
        for jp in range(k):
            Bs[jp][z] = acc_b[jp]
    A = rescale_by(A, F.P.p, primes)
    out_b = []
    for jp in range(k):
        Bj = rescale_by(Bs[jp], F.P.p, primes)
        out_b.append({q: (chunks[jp][1][q] + Bj[q]) % q for q in primes})
    return A, out_b


def format_switch(F: FSKeys, ct: Dict[int, np.ndarray], d3: int) -> Dict[int, np.ndarray]:
    """Transmission ciphertexts -> the CCMM query ciphertext XT per query prime i < level:
    d3 x (d2 + N_Q), row c = [b_c (the k chunks' b, first d2 coefficients) | a_c]."""
    P, lvl = F.P, F.level
    primes = F.primes_in()
    k = P.k
    ql = P.q[lvl]
    keep = primes[:lvl]
    XT = {i: np.zeros((d3, P.K), dtype=np.int64) for i in range(lvl)}
    for c in range(d3):
        chunks = [ring_switch(F, ct, c * k + j) for j in range(k)]
        a, bs = convert(F, chunks)
        a_l = rescale_by(a, ql, keep)
        b_l = [rescale_by(bj, ql, keep) for bj in bs]
        for i, q in enumerate(keep):
            bcat = np.concatenate([b_l[j][q] for j in range(k)])[:P.d2]
            XT[i][c] = np.concatenate([bcat, a_l[q]])
    return XT
