"""Pins of the oracle's encryption and CCMM against invariants the paper fixes.

* Dec(a, b) = a*sk + b recovers scale*m up to the sampled error (Section 2.2.2),
  with the secret products taken by a route independent of the oracle's
  Neg-matrix (numpy.polymul folded mod X^n + 1, and the conjugate-secret form
  of M_DB S_Q).
* The CCMM result decrypts to the masked inner products of Section 2.1.3,
  computed by brute-force popcount, within 0.25 on every pair, and the
  threshold decisions agree.
* Special cases: unit-vector query columns return database columns; an
  all-zero query decrypts to zero.
"""
import numpy as np
import pytest

import hfe_synth as S
from oracle import ckks as OC
from oracle import iris as OI
from oracle import prng

from oracle_cases import DB_SEED, KEY_SEED, Q_SEED, case, params_for


def _fold(s, a):
    n = len(s)
    full = np.polymul(np.asarray(s, dtype=object)[::-1], np.asarray(a, dtype=object)[::-1])[::-1]
    full = list(full) + [0] * (2 * n - len(full))
    return np.array([int(full[t]) - int(full[t + n]) for t in range(n)], dtype=object)


def _centered(x, q):
    x = int(x) % q
    return x - q if x > q // 2 else x


@pytest.mark.parametrize("name", [S.TINY_MULTI.name])
def test_query_encryption_decrypts_to_delta_m_plus_small_error(name):
    c = case(name)
    P = c.P
    delta = P.delta(c.w.level)
    for i in range(c.w.level):
        qi = P.q[i]
        for col in range(c.m_q.shape[0]):
            b = c.XT[i][col, :P.d2]
            a = c.XT[i][col, P.d2:]
            for j in range(P.k):
                sa = _fold(c.keys.s[j], a)
                lo, hi = j * P.n_q, min((j + 1) * P.n_q, P.d2)
                for t in range(lo, hi):
                    e = _centered(int(b[t]) + int(sa[t - lo]) - delta * int(c.m_q[col, t]), qi)
                    assert -19 <= e <= 19


@pytest.mark.parametrize("name", [S.TINY_MULTI.name])
def test_db_encryption_decrypts_to_p_times_plaintext(name):
    c = case(name)
    P = c.P
    n = P.n_q
    # T = M_DB S_Q through the conjugate secret s~(X) = s(X^-1): row i of T is the sum over
    # chunks j of s~_j * (chunk j of row i).
    T = np.zeros((c.m_db.shape[0], n), dtype=object)
    for j in range(P.k):
        s = c.keys.s[j]
        st = np.array([s[0]] + [-s[n - k] for k in range(1, n)])
        lo, hi = j * n, min((j + 1) * n, P.d2)
        for i in range(c.m_db.shape[0]):
            chunk = np.zeros(n, dtype=np.int64)
            chunk[:hi - lo] = c.m_db[i, lo:hi]
            T[i] += _fold(st, chunk)
    plain = np.concatenate([c.m_db.astype(object), T], axis=1)
    rng = np.random.default_rng(0)
    cols = sorted(rng.choice(P.K, 12, replace=False).tolist()) + [0, P.d2 - 1, P.d2, P.K - 1]
    for pid, prime in OC.prime_ids(P, len(P.q)):
        D = c.D[pid]
        for col in cols:
            a = D[:P.n_db, col]
            for j in range(P.k_db):
                sa = _fold(c.keys.s_db[j], a)
                for i in range(j * P.n_db, min((j + 1) * P.n_db, c.m_db.shape[0])):
                    e = _centered(int(D[P.n_db + i, col]) + int(sa[i - j * P.n_db])
                                  - P.p * int(plain[i, col]), prime)
                    assert -19 <= e <= 19


@pytest.mark.parametrize("name", [S.TINY.name, S.TINY_MULTI.name])
def test_ccmm_decrypts_to_popcount_inner_products(name):
    c = case(name)
    assert np.array_equal(c.ip, c.ip_true)
    err = max(abs(float(c.v[a][b]) - int(c.ip_true[a, b]))
              for a in range(len(c.v)) for b in range(c.rows))
    assert err <= 0.25
    dec = OI.decide(c.ip, c.overlap)
    assert np.array_equal(dec, OI.decide(c.ip_true, c.overlap))
    for pl in S.planted_for(c.w):
        col = pl.eye * c.w.n_shifts + list(S.default_shifts(c.w.n_shifts)).index(pl.shift)
        assert dec[col, pl.db_row - c.row0]


def test_ccmm_on_a_row_shard_matches_the_full_result():
    full = case(S.TINY_MULTI.name)
    part = case(S.TINY_MULTI.name, 100, 60)
    n = full.P.n_db
    for i in range(full.w.level):
        assert np.array_equal(part.out[i][:, :n], full.out[i][:, :n])
        assert np.array_equal(part.out[i][:, n:], full.out[i][:, n + 100:n + 160])
    assert np.array_equal(part.ip, full.ip[:, 100:160])


def test_unit_vector_and_zero_queries():
    w = S.TINY_MULTI
    P = params_for(w)
    c = case(w.name)
    d2 = P.d2
    ks = [0, 5, 511, 512, 1023]
    mq = np.zeros((len(ks) + 1, d2), dtype=np.int8)
    for r, k in enumerate(ks):
        mq[r, k] = 1 if r % 2 == 0 else -1
    XT = OC.encrypt_query(c.keys, mq, w.level, Q_SEED + 1)
    out = OC.ccmm(P, c.D, XT, w.level, 0, w.d1)
    v, ip = OC.decrypt(c.keys, out, w.level, 0, w.d1)
    for r, k in enumerate(ks):
        sign = 1 if r % 2 == 0 else -1
        assert np.array_equal(ip[r], sign * c.m_db[:, k].astype(np.int64))
    assert np.all(ip[len(ks)] == 0)


def test_ccmm_invariant_before_rescale():
    """B_pre + S_DB A_pre = p Delta M_DB M_Q + small (mod Q p), on the big integers."""
    c = case(S.TINY_MULTI.name)
    P = c.P
    lvl = c.w.level
    C = OC.ccmm_pre_rescale(P, c.D, c.XT, lvl, 0, c.w.d1)
    ids = OC.prime_ids(P, lvl)
    moduli = [m for _, m in ids]
    Qp = P.Q(lvl) * P.p
    delta = P.delta(lvl)
    big = {(r, col): OC.crt([int(C[pid][r, col]) for pid, _ in ids], moduli)
           for r in range(P.n_db + c.w.d1) for col in range(c.m_q.shape[0])}
    S_rows = OC.s_db_rows(c.keys, range(c.w.d1))
    for col in range(c.m_q.shape[0]):
        a_pre = [big[(v, col)] for v in range(P.n_db)]
        for i in range(0, c.w.d1, 17):
            y = big[(P.n_db + i, col)] + sum(int(S_rows[i, v]) * a_pre[v] for v in range(P.n_db))
            noise = OC.centered(y - P.p * delta * int(c.ip_true[col, i]), Qp)
            assert abs(noise) < P.p * delta // 8


def test_single_entry_functions_match_the_full_oracle():
    """The sampled-entry evaluations used at large sizes agree with the full-matrix oracle."""
    c = case(S.TINY_MULTI.name)
    P = c.P
    for pid, prime in OC.prime_ids(P, len(P.q)):
        for r, col in [(0, 0), (5, 1000), (P.n_db, 3), (P.n_db + 255, P.K - 1), (P.n_db + 130, P.d2 + 7)]:
            assert OC.db_entry(c.keys, c.m_db, DB_SEED, pid, prime, r, col) == c.D[pid][r, col]
    for col in (0, 3):
        qc = OC.query_column(c.keys, c.m_q[col], c.w.level, Q_SEED, col)
        for i in range(c.w.level):
            assert np.array_equal(qc[i], c.XT[i][col])
    for r, col in [(3, 0), (P.n_db + 17, 1), (P.n_db + 255, 3)]:
        drow = {pid: c.D[pid][r] for pid, _ in OC.prime_ids(P, c.w.level)}
        xc = {i: c.XT[i][col] for i in range(c.w.level)}
        assert OC.ccmm_entry(P, drow, xc, c.w.level) == [c.out[i][col, r] for i in range(c.w.level)]
    s = c.keys.s[0]
    a = np.arange(P.n_q) * 7919 % 1000
    from oracle.ring import neg_matrix
    assert np.array_equal(OC.negmul_vec(s, a), neg_matrix(s) @ a)


def test_block_functions_match_the_full_oracle():
    """The row, column and grid evaluations used at large sizes (db_rows, query_columns, lift_mod,
    ccmm_entries, s_q_columns) agree with the full-matrix oracle on the mid workload, whose secret
    stacks have three chunks with a truncated last one; chunk sizes of the row evaluation are chosen
    so that the chunks end inside and on the ring boundaries."""
    c = case(S.MID.name)
    P = c.P
    SQ = OC.s_q_matrix(c.keys)
    assert np.array_equal(OC.s_q_columns(c.keys, 0, P.n_q), SQ)
    assert np.array_equal(OC.s_q_columns(c.keys, 100, 317), SQ[:, 100:317])
    rows = [0, 1, P.n_db - 1, P.n_db, P.n_db + 1, P.n_db + 255, P.n_db + 256, P.n_db + c.w.d1 - 1]
    for pid, prime in OC.prime_ids(P, len(P.q)):
        for chunk in (100, 512):
            assert np.array_equal(OC.db_rows(c.keys, c.m_db, DB_SEED, pid, prime, rows, chunk=chunk), c.D[pid][rows])
    cols = [0, 5, c.w.d3 - 1, 130]
    qc = OC.query_columns(c.keys, c.m_q[cols], cols, c.w.level, Q_SEED)
    for i in range(c.w.level):
        assert np.array_equal(qc[i], c.XT[i][cols])
    L = OC.lift_query(P, {i: c.XT[i][cols] for i in range(c.w.level)}, c.w.level)
    for _, prime in OC.prime_ids(P, c.w.level):
        lm = OC.lift_mod(P, {i: c.XT[i][cols] for i in range(c.w.level)}, c.w.level, prime)
        assert lm.tolist() == [[v % prime for v in col] for col in L]
    out_rows = rows[:3] + [P.n_db + 17, P.n_db + 699]
    d = {pid: c.D[pid][out_rows] for pid, _ in OC.prime_ids(P, c.w.level)}
    e = OC.ccmm_entries(P, d, qc, c.w.level)
    for i in range(c.w.level):
        assert np.array_equal(e[i], c.out[i][np.ix_(cols, out_rows)])


def test_uniform_columns_equal_the_oracle_philox():
    """The bulk generator (numpy's Philox bit generator) gives the elements of uniform_matrix, on
    columns 0 (whose counter wraps below zero) and beyond, with and without the rejection path."""
    from oracle.params import ntt_primes
    q = ntt_primes(1)[0]
    for qq in (q, (1 << 63) + 25):
        A = prng.uniform_matrix(11, prng.DBA, 3, 41, 9, qq)
        for c0, c1 in ((0, 9), (4, 7)):
            assert np.array_equal(prng.uniform_columns(11, prng.DBA, 3, 41, c0, c1, qq), A[:, c0:c1])


def test_share_golden_samples_agree_with_the_single_entry_oracle():
    """Entries of golden/share_samples.json (written by make_share_samples.py with the row, column and
    grid functions) recomputed by the single-entry functions db_entry and ccmm_entry."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "share_samples.json")) as f:
        g = json.load(f)
    w = S.PAPER_SHARE
    assert g["workload"] == w.name
    P = params_for(w)
    keys = OC.keygen(P, g["seeds"]["keys"])
    inp = S.make_inputs(w)
    m_db = OI.ternary(inp["db_codes"], inp["db_masks"])
    ids = OC.prime_ids(P, len(P.q))
    rows, kcols = g["rows"], g["db_cols"]
    for z, a, b in ((0, 0, 0), (3, 31, 31), (1, 20, 5), (2, 17, 30), (3, 16, 12), (0, 24, 9)):
        pid, prime = ids[z]
        assert OC.db_entry(keys, m_db, g["seeds"]["db"], pid, prime, rows[a], kcols[b]) == g["db"][z][a][b]
    qc, qm = OI.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    m_q = OI.ternary(qc, qm)
    kk = np.arange(P.K)
    for a, b in ((0, 0), (7, 63)):              # A-part rows: whole rows of uniform elements
        r, col = rows[a], g["cols"][b]
        xt = OC.query_column(keys, m_q[col], w.level, g["seeds"]["query"], col)
        d_row = {pid: prng.uniform_mod(g["seeds"]["db"], prng.DBA, pid, np.full(P.K, r), kk, prime)
                 for pid, prime in OC.prime_ids(P, w.level)}
        assert OC.ccmm_entry(P, d_row, xt, w.level) == [g["result"][i][b][a] for i in range(w.level)]
