"""Keys, encryption, the encrypted matrix product (CCMM), rescale, decryption (oracle).

Notation (Section 2.3 and Section 6.3 of the paper, with the readings listed
in the design notes):
  M_DB  d1 x d2 ternary matrix, one database code per row
  M_Q   d2 x d3 ternary matrix, one query vector per column
  s_j   query secrets in R_{N_Q}, j < k = ceil(d2 / N_Q);   S_Q  = stack Neg(s_j), first d2 rows
  s'_j  database secrets in R_{N_DB}, j < k';               S_DB = stack Neg(s'_j), first d1 rows
  Decryption is a * sk + b (Section 2.2.2), so encryption sets b = -S a + scale * m + e.

Query ciphertext (MSRLWE, modulus Q = q_0 ... q_{l-1}):
  A_Q  (N_Q x d3) uniform,  B_Q = -S_Q A_Q + Delta M_Q + E_Q  (d2 x d3)
Database ciphertext (modulus Q_L p):
  T = M_DB S_Q (exact integers),  A = [A1 | A2]  (N_DB x (d2 + N_Q)) uniform,
  B = [B1 | B2] = -S_DB A + p [M_DB | T] + [E1 | E2]
  stored per prime as D = [[A], [B]]: (N_DB + d1) x (d2 + N_Q)
CCMM (the four plaintext products of Section 2.3, written as one product per
prime):  X = [L(B_Q); L(A_Q)] where L lifts a residue vector mod Q to its
centered representative; C = D X mod Q p; result = RS_p(C) mod Q where
RS_p(x) = floor(x / p + 1/2) (Section 2.2.4 with the rounding of Section 1.1).
Then B_out + S_DB A_out = Delta M_DB M_Q + small noise (mod Q).

Residue arrays are int64 with entries in [0, prime).  Every function below
keeps to the plain definition; the GPU library never calls into this module.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import prng
from .params import Params
from .ring import imatmul, modmatmul, neg_matrix


@dataclasses.dataclass
class Keys:
    params: Params
    seed: int
    s: np.ndarray       # (k, N_Q) ternary query secrets
    s_db: np.ndarray    # (k', N_DB) ternary database secrets


def keygen(params: Params, seed: int) -> Keys:
    s = np.stack([prng.ternary(seed, prng.QSEC, j, params.n_q) for j in range(params.k)])
    s_db = np.stack([prng.ternary(seed, prng.DBSEC, j, params.n_db) for j in range(params.k_db)])
    return Keys(params, seed, s, s_db)


def s_q_matrix(keys: Keys) -> np.ndarray:
    """S_Q: d2 x N_Q, the stack of Neg(s_j) truncated to d2 rows."""
    P = keys.params
    # only the first d2 rows of the stack exist: secret j contributes min(N_Q, d2 - j N_Q) rows
    return np.concatenate([neg_matrix(keys.s[j], min(P.n_q, P.d2 - j * P.n_q)) for j in range(P.k)], axis=0)


def s_db_rows(keys: Keys, rows: Sequence[int]) -> np.ndarray:
    """Selected rows of S_DB (stack of Neg(s'_j)), as an int64 matrix (len(rows) x N_DB)."""
    n = keys.params.n_db
    out = np.empty((len(rows), n), dtype=np.int64)
    for r, i in enumerate(rows):
        j, t = divmod(int(i), n)
        s = keys.s_db[j]
        v = np.arange(n)
        d = t - v
        out[r] = np.where(d >= 0, s[d % n], -s[d % n])
    return out


def prime_ids(params: Params, level: int) -> List[Tuple[int, int]]:
    """(stream id, prime) for the query primes of a level and the special prime."""
    return [(i, params.q[i]) for i in range(level)] + [(prng.P_ID, params.p)]


# ---------------------------------------------------------------- encryption

def encrypt_db_with(P: Params, SQ: np.ndarray, SDB: np.ndarray, m_db: np.ndarray,
                    A: Dict[int, np.ndarray], E: np.ndarray) -> Dict[int, np.ndarray]:
    """Database ciphertext from explicit randomness.

    SQ: d2 x N_Q query secret matrix; SDB: d1 x N_DB database secret rows;
    A[pid]: N_DB x K uniform residues per prime; E: d1 x K integer errors.
    Returns D per prime stream id: (N_DB + d1) x K with D = [[A], [B]] and
    B = -S_DB A + p [M_DB | M_DB S_Q] + E  (mod prime).
    """
    T = imatmul(m_db.astype(np.int64), SQ)                              # d1 x N_Q, exact
    plain = np.concatenate([m_db.astype(np.int64), T], axis=1)          # [M_DB | T]
    out = {}
    for pid, prime in prime_ids(P, len(P.q)):
        B = (-imatmul(SDB, A[pid]) + (P.p % prime) * plain + E) % prime
        out[pid] = np.concatenate([A[pid], B], axis=0)
    return out


def encrypt_db(keys: Keys, m_db: np.ndarray, seed: int) -> Dict[int, np.ndarray]:
    """Database ciphertext residues D per prime stream id: (N_DB + d1) x (d2 + N_Q)."""
    P = keys.params
    d1, d2 = m_db.shape
    assert d2 == P.d2 and d1 <= P.max_db_rows
    A = {pid: prng.uniform_matrix(seed, prng.DBA, pid, P.n_db, P.K, prime)
         for pid, prime in prime_ids(P, len(P.q))}
    E = prng.gaussian_matrix(seed, prng.DBE, 0, d1, P.K)
    return encrypt_db_with(P, s_q_matrix(keys), s_db_rows(keys, range(d1)), m_db, A, E)


def encrypt_query_with(P: Params, SQ: np.ndarray, m_q_rows: np.ndarray, level: int,
                       A: Dict[int, np.ndarray], E: np.ndarray) -> Dict[int, np.ndarray]:
    """Query ciphertext from explicit randomness.

    A[i]: N_Q x d3 uniform residues mod q_i; E: d2 x d3 integer errors.
    Returns XT per query prime i: d3 x (d2 + N_Q), row c = [b_c | a_c] with
    b_c = -S_Q a_c + Delta m_c + e_c  (mod q_i).
    """
    delta = P.delta(level)
    MQ = m_q_rows.astype(np.int64).T                                     # d2 x d3
    out = {}
    for i in range(level):
        qi = P.q[i]
        B = (-imatmul(SQ, A[i]) + (delta % qi) * MQ + E) % qi             # d2 x d3
        out[i] = np.concatenate([B.T, A[i].T], axis=1)
    return out


def encrypt_query(keys: Keys, m_q_rows: np.ndarray, level: int, seed: int) -> Dict[int, np.ndarray]:
    """Query ciphertext per query prime id i < level: XT (d3 x (d2 + N_Q)) = [b_c | a_c] per row c."""
    P = keys.params
    d3, d2 = m_q_rows.shape
    assert d2 == P.d2 and 1 <= level <= len(P.q)
    A = {i: prng.uniform_matrix(seed, prng.QA, i, P.n_q, d3, P.q[i]) for i in range(level)}
    E = prng.gaussian_matrix(seed, prng.QE, 0, d2, d3)
    return encrypt_query_with(P, s_q_matrix(keys), m_q_rows, level, A, E)


# ---------------------------------------------------------------- CRT helpers

def crt(residues: Sequence[int], moduli: Sequence[int]) -> int:
    """The unique x in [0, prod moduli) with x = r_i mod m_i."""
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def centered(x: int, M: int) -> int:
    """Representative of x mod M in (-M/2, M/2] (M odd: in (-M/2, M/2))."""
    x %= M
    return x - M if x > M // 2 else x


# ---------------------------------------------------------------- CCMM

def lift_query(P: Params, XT: Dict[int, np.ndarray], level: int) -> List[List[int]]:
    """L(x): centered representative mod Q of every query residue vector (Python ints)."""
    moduli = [P.q[i] for i in range(level)]
    Q = P.Q(level)
    d3, K = XT[0].shape
    return [[centered(crt([int(XT[i][c, k]) for i in range(level)], moduli), Q) for k in range(K)]
            for c in range(d3)]


def ccmm_pre_rescale(P: Params, D: Dict[int, np.ndarray], XT: Dict[int, np.ndarray], level: int,
                     row0: int, rows: int) -> Dict[int, np.ndarray]:
    """C = D_sel X mod prime for each prime of the level and p: (N_DB + rows) x d3."""
    L = lift_query(P, XT, level)
    sel = np.concatenate([np.arange(P.n_db), P.n_db + row0 + np.arange(rows)])
    out = {}
    for pid, prime in prime_ids(P, level):
        X = np.array([[v % prime for v in col] for col in L], dtype=np.int64).T   # K x d3
        out[pid] = modmatmul(D[pid][sel], X, prime)
    return out


def rescale_p(x: int, p: int, Q: int) -> int:
    """RS_p(x) = floor(x / p + 1/2) mod Q for an integer x (p odd: no ties)."""
    return ((2 * x + p) // (2 * p)) % Q


def ccmm(P: Params, D: Dict[int, np.ndarray], XT: Dict[int, np.ndarray], level: int,
         row0: int, rows: int) -> Dict[int, np.ndarray]:
    """Result ciphertext per query prime i: (d3 x (N_DB + rows)) = [A_out | B_out] per column."""
    C = ccmm_pre_rescale(P, D, XT, level, row0, rows)
    ids = prime_ids(P, level)
    moduli = [m for _, m in ids]
    Q = P.Q(level)
    R, d3 = C[ids[0][0]].shape
    res = {i: np.empty((d3, R), dtype=np.int64) for i in range(level)}
    for r in range(R):
        for c in range(d3):
            x = crt([int(C[pid][r, c]) for pid, _ in ids], moduli)
            y = rescale_p(x, P.p, Q)
            for i in range(level):
                res[i][c, r] = y % P.q[i]
    return res


# ---------------------------------------------------------------- decryption

def decrypt(keys: Keys, out: Dict[int, np.ndarray], level: int, row0: int, rows: int
            ) -> Tuple[List[List[Fraction]], np.ndarray]:
    """(v, IP): v = centered(B_out + S_DB A_out mod Q) / Delta as Fractions; IP = floor(v + 1/2)."""
    P = keys.params
    Q = P.Q(level)
    delta = P.delta(level)
    S = s_db_rows(keys, range(row0, row0 + rows))                         # rows x N_DB
    y = {}
    for i in range(level):
        A_out = out[i][:, :P.n_db]
        B_out = out[i][:, P.n_db:]
        y[i] = (B_out + imatmul(A_out, S.T)) % P.q[i]                     # d3 x rows
    d3 = out[0].shape[0]
    v = [[Fraction(0)] * rows for _ in range(d3)]
    ip = np.empty((d3, rows), dtype=np.int64)
    moduli = [P.q[i] for i in range(level)]
    for c in range(d3):
        for r in range(rows):
            yc = centered(crt([int(y[i][c, r]) for i in range(level)], moduli), Q)
            v[c][r] = Fraction(yc, delta)
            ip[c, r] = (2 * yc + delta) // (2 * delta)
    return v, ip


# ---------------------------------------------------------------- single entries (large sizes)
# The functions below evaluate the same definitions one entry or one column at a time, for
# workloads too large to materialise (checks on sampled entries).

def negmul_vec(s: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Schoolbook s * a in Z[X]/(X^n + 1): sum over u of s_u X^u a, where X^u a shifts a up by
    u places and negates the u coefficients that wrap past degree n - 1."""
    n = len(a)
    a = np.asarray(a, dtype=np.int64)
    out = np.zeros(n, dtype=np.int64)
    for u in np.nonzero(s)[0]:
        shifted = np.roll(a, u)
        shifted[:u] = -shifted[:u]
        out += int(s[u]) * shifted
    return out


def s_q_column(keys: Keys, v: int) -> np.ndarray:
    """Column v of S_Q (d2 entries): rows of chunk j are Neg(s_j)[t][v]."""
    P = keys.params
    n = P.n_q
    t = np.arange(P.d2)
    j, tt = t // n, t % n
    d = tt - v
    s = keys.s[j, d % n]
    return np.where(d >= 0, s, -s).astype(np.int64)


def db_entry(keys: Keys, m_db: np.ndarray, seed: int, pid: int, prime: int, r: int, c: int) -> int:
    """D[r][c] mod prime of the database ciphertext (r < N_DB: A-part, else code row r - N_DB)."""
    P = keys.params
    if r < P.n_db:
        return int(prng.uniform_mod(seed, prng.DBA, pid, [r], [c], prime)[0])
    i = r - P.n_db
    a_c = prng.uniform_mod(seed, prng.DBA, pid, np.arange(P.n_db), c, prime)
    sa = int(imatmul(s_db_rows(keys, [i]), a_c.reshape(-1, 1))[0, 0])
    if c < P.d2:
        plain = int(m_db[i, c])
    else:
        plain = int(imatmul(m_db[i].astype(np.int64).reshape(1, -1),
                            s_q_column(keys, c - P.d2).reshape(-1, 1))[0, 0])
    e = int(prng.gaussian(seed, prng.DBE, 0, [i], [c])[0])
    return (-sa + P.p * plain + e) % prime


def query_column(keys: Keys, m_q_row: np.ndarray, level: int, seed: int, c: int) -> Dict[int, np.ndarray]:
    """Row c of XT per query prime i: [b_c | a_c] of query column c (m_q_row = its d2 entries)."""
    P = keys.params
    n = P.n_q
    delta = P.delta(level)
    e = prng.gaussian(seed, prng.QE, 0, np.arange(P.d2), c)
    out = {}
    for i in range(level):
        qi = P.q[i]
        a = prng.uniform_mod(seed, prng.QA, i, np.arange(n), c, qi)
        b = np.empty(P.d2, dtype=np.int64)
        for j in range(P.k):
            lo, hi = j * n, min((j + 1) * n, P.d2)
            sa = negmul_vec(keys.s[j], a)
            b[lo:hi] = (-sa[:hi - lo] + (delta % qi) * m_q_row[lo:hi].astype(np.int64) + e[lo:hi]) % qi
        out[i] = np.concatenate([b, a])
    return out


def ccmm_entry(P: Params, d_row: Dict[int, List[int]], xt_col: Dict[int, np.ndarray], level: int) -> List[int]:
    """Result residues (per query prime) of one output entry: RS_p of sum_k D[r][k] L(x)[k],
    given row r of D per prime stream id and the query column's residues."""
    moduli = [P.q[i] for i in range(level)]
    Q = P.Q(level)
    K = len(xt_col[0])
    L = [centered(crt([int(xt_col[i][k]) for i in range(level)], moduli), Q) for k in range(K)]
    ids = prime_ids(P, level)
    res = [sum(int(d_row[pid][k]) * (L[k] % prime) for k in range(K)) % prime for pid, prime in ids]
    x = crt(res, [m for _, m in ids])
    y = rescale_p(x, P.p, Q)
    return [y % qi for qi in moduli]


# ---------------------------------------------------------------- row and column blocks (large sizes)
# Whole database rows, selected query columns and grids of result entries, evaluated from the same
# definitions as the full-matrix functions above, for workloads whose full matrices do not fit.

def s_q_columns(keys: Keys, v0: int, v1: int) -> np.ndarray:
    """Columns v0 .. v1 - 1 of S_Q (d2 x (v1 - v0)): row t of chunk j is Neg(s_j)[t - j N_Q]."""
    P = keys.params
    n = P.n_q
    t = np.arange(P.d2)[:, None]
    v = np.arange(v0, v1)[None, :]
    d = t % n - v
    s = keys.s[t // n, d % n]
    return np.where(d >= 0, s, -s).astype(np.int64)


def db_rows(keys: Keys, m_db: np.ndarray, seed: int, pid: int, prime: int, rows: Sequence[int],
            chunk: int = 512) -> np.ndarray:
    """Rows `rows` of D mod prime ((len(rows) x K) int64), as encrypt_db defines them: A rows are the
    uniform elements; B row i = -S_DB[i] A + p [M_DB[i] | M_DB[i] S_Q] + E[i], with A and S_Q taken
    chunk columns at a time."""
    P = keys.params
    rows = [int(r) for r in rows]
    K = P.K
    kk = np.arange(K)
    out = np.empty((len(rows), K), dtype=np.int64)
    for idx, r in enumerate(rows):
        if r < P.n_db:
            out[idx] = prng.uniform_mod(seed, prng.DBA, pid, np.full(K, r), kk, prime)
    bidx = [idx for idx, r in enumerate(rows) if r >= P.n_db]
    if not bidx:
        return out
    b = [rows[idx] - P.n_db for idx in bidx]
    M = m_db[b].astype(np.int64)                                            # nb x d2
    plain = np.empty((len(b), K), dtype=np.int64)
    plain[:, :P.d2] = M
    for v0 in range(0, P.n_q, chunk):
        v1 = min(P.n_q, v0 + chunk)
        plain[:, P.d2 + v0:P.d2 + v1] = imatmul(M, s_q_columns(keys, v0, v1))
    S = s_db_rows(keys, b)                                                  # nb x N_DB
    SA = np.empty((len(b), K), dtype=np.int64)
    for c0 in range(0, K, chunk):
        c1 = min(K, c0 + chunk)
        SA[:, c0:c1] = imatmul(S, prng.uniform_columns(seed, prng.DBA, pid, P.n_db, c0, c1, prime))
    E = prng.gaussian(seed, prng.DBE, 0, np.repeat(b, K), np.tile(kk, len(b))).reshape(len(b), K)
    out[bidx] = (-SA + (P.p % prime) * plain + E) % prime
    return out


def query_columns(keys: Keys, m_q_rows: np.ndarray, cols: Sequence[int], level: int, seed: int
                  ) -> Dict[int, np.ndarray]:
    """Rows `cols` of XT per query prime i ((len(cols) x K)): encrypt_query restricted to the query
    columns cols, whose d2 entries are the rows of m_q_rows."""
    P = keys.params
    cols = np.asarray(cols, dtype=np.uint64)
    n = len(cols)
    t = np.arange(P.n_q, dtype=np.uint64)
    A = {i: prng.uniform_mod(seed, prng.QA, i, np.repeat(t, n), np.tile(cols, P.n_q), P.q[i]).reshape(P.n_q, n)
         for i in range(level)}
    tt = np.arange(P.d2, dtype=np.uint64)
    E = prng.gaussian(seed, prng.QE, 0, np.repeat(tt, n), np.tile(cols, P.d2)).reshape(P.d2, n)
    return encrypt_query_with(P, s_q_matrix(keys), m_q_rows, level, A, E)


def lift_mod(P: Params, XT: Dict[int, np.ndarray], level: int, prime: int) -> np.ndarray:
    """L(x) mod prime for every query residue vector (int64, the shape of XT[0]): the CRT value of
    the residues mod Q (sum of x_i (Q/q_i) ((Q/q_i)^-1 mod q_i), mod Q), centered, reduced mod prime;
    the arithmetic of crt and centered on Python integers held in object arrays."""
    moduli = [P.q[i] for i in range(level)]
    Q = P.Q(level)
    acc = np.zeros(XT[0].shape, dtype=object)
    for i, m in enumerate(moduli):
        Mi = Q // m
        acc = acc + XT[i].astype(object) * (Mi * pow(Mi, -1, m))
    acc = acc % Q
    acc = np.where(acc > Q // 2, acc - Q, acc)
    return (acc % prime).astype(np.int64)


def ccmm_entries(P: Params, d_rows: Dict[int, np.ndarray], xt_cols: Dict[int, np.ndarray], level: int
                 ) -> Dict[int, np.ndarray]:
    """Result residues per query prime i ((n_cols x n_rows)) of the entries (row, column) of a grid:
    d_rows[pid] holds the grid's rows of D per prime stream id, xt_cols[i] its query columns' rows of
    XT.  Each entry is RS_p of the exact product of its row and the lifted column, as in ccmm."""
    ids = prime_ids(P, level)
    moduli = [m for _, m in ids]
    Q = P.Q(level)
    C = {pid: modmatmul(d_rows[pid], lift_mod(P, xt_cols, level, prime).T, prime) for pid, prime in ids}
    nr, nc = C[ids[0][0]].shape
    res = {i: np.empty((nc, nr), dtype=np.int64) for i in range(level)}
    for r in range(nr):
        for c in range(nc):
            y = rescale_p(crt([int(C[pid][r, c]) for pid, _ in ids], moduli), P.p, Q)
            for i in range(level):
                res[i][c, r] = y % P.q[i]
    return res
