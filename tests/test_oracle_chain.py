"""Pins of the oracle's CCMM over the n^2 modulus chain (oracle/chain.py, Section 6.3).

Each check rests on something other than the oracle's own formulas: the bases by trial division,
encryption by the decryption equation with the secret products taken by numpy.polymul folded mod
X^n + 1 (T through the conjugate secret), the whole CCMM by the brute-force popcount inner products,
the product before the rescale by the plaintext it must carry on the big integers, and the rescale by
Fraction rounding with a composite odd divisor.
"""
from fractions import Fraction

import numpy as np
import pytest

import hfe_synth as S
from oracle import chain as OCH
from oracle import ckks as OC
from oracle import iris as OI

from oracle_cases import chain_case

W = S.CHAIN_TINY


def _fold(s, a):
    """s * a in Z[X]/(X^n + 1) by numpy.polymul on Python integers, folded."""
    n = len(s)
    full = np.polymul(np.array(s[::-1], dtype=object), np.array([int(x) for x in a[::-1]], dtype=object))[::-1]
    out = np.zeros(n, dtype=object)
    for i, v in enumerate(full):
        if i < n:
            out[i] += v
        else:
            out[i - n] -= v
    return out


def _centered(x, m):
    x = int(x) % m
    return x - m if x > m // 2 else x


def test_chain_bases_are_the_primes_from_127_to_253():
    trial = [n for n in range(127, 254) if all(n % d for d in range(2, int(n ** 0.5) + 1))]
    assert sorted(OCH.CHAIN_BASES) == trial
    assert len(trial) == 24                                # 48 int8 planes (Section 6.3)
    C = OCH.make_chain_params(9, 9, 7, 3, 512, 256)
    mods = C.q_mods(7) + C.p_mods
    for i in range(len(mods)):
        for j in range(i):
            assert np.gcd(mods[i], mods[j]) == 1
    assert C.P % 2 == 1 and C.P.bit_length() >= 36       # room for the rescale's noise division


@pytest.mark.parametrize("level", [7, 5])
def test_chain_query_encryption_decrypts_to_delta_m_plus_small_error(level):
    c = chain_case(W.name, level)
    C = c.C
    delta = C.delta(level)
    for n in C.q_bases[:level]:
        m = n * n
        for col in range(c.m_q.shape[0]):
            b, a = c.XT[n][col, :C.d2], c.XT[n][col, C.d2:]
            for j in range(-(-C.d2 // C.n_q)):
                sa = _fold(c.keys.s[j], a)
                lo, hi = j * C.n_q, min((j + 1) * C.n_q, C.d2)
                for t in range(lo, hi):
                    assert -19 <= _centered(int(b[t]) + int(sa[t - lo]) - delta * int(c.m_q[col, t]), m) <= 19


def test_chain_db_encryption_decrypts_to_P_times_plaintext():
    c = chain_case(W.name)
    C = c.C
    n_q = C.n_q
    T = np.zeros((c.m_db.shape[0], n_q), dtype=object)
    for j in range(-(-C.d2 // n_q)):
        s = c.keys.s[j]
        st = np.array([s[0]] + [-s[n_q - k] for k in range(1, n_q)])
        lo, hi = j * n_q, min((j + 1) * n_q, C.d2)
        for i in range(c.m_db.shape[0]):
            chunk = np.zeros(n_q, dtype=np.int64)
            chunk[:hi - lo] = c.m_db[i, lo:hi]
            T[i] += _fold(st, chunk)
    plain = np.concatenate([c.m_db.astype(object), T], axis=1)
    rng = np.random.default_rng(0)
    cols = sorted(rng.choice(C.K, 8, replace=False).tolist()) + [0, C.d2 - 1, C.d2, C.K - 1]
    for n in C.all_bases():
        m = n * n
        D = c.D[n]
        for col in cols:
            sa = _fold(c.keys.s_db[0], D[:C.n_db, col])
            for i in range(c.m_db.shape[0]):
                e = _centered(int(D[C.n_db + i, col]) + int(sa[i]) - C.P * int(plain[i, col]), m)
                assert -19 <= e <= 19


@pytest.mark.parametrize("level", [7, 5])
def test_chain_ccmm_decrypts_to_popcount_inner_products(level):
    c = chain_case(W.name, level)
    assert np.array_equal(c.ip, c.ip_true)
    err = max(abs(float(c.v[a][b]) - int(c.ip_true[a, b])) for a in range(len(c.v)) for b in range(W.d1))
    assert err <= 0.25
    dec = OI.decide(c.ip, c.overlap)
    for pl in S.planted_for(c.w):
        col = pl.eye * c.w.n_shifts + list(S.default_shifts(c.w.n_shifts)).index(pl.shift)
        assert dec[col, pl.db_row]


def test_chain_product_before_rescale_carries_P_delta_times_the_plaintext_product():
    """B_pre + S_DB A_pre = P Delta M_DB M_Q + small (mod Q P), on the big integers."""
    c = chain_case(W.name)
    C, lvl = c.C, c.level
    pre = OCH.ccmm_pre_rescale(C, c.D, c.XT, lvl, 0, W.d1)
    bases = list(C.q_bases[:lvl]) + list(C.p_bases)
    moduli = [n * n for n in bases]
    QP = C.Q(lvl) * C.P
    delta = C.delta(lvl)
    S_rows = OC.s_db_rows(c.keys, range(W.d1))
    for col in range(c.m_q.shape[0]):
        a_pre = [OC.crt([int(pre[n][v, col]) for n in bases], moduli) for v in range(C.n_db)]
        for i in range(0, W.d1, 23):
            b = OC.crt([int(pre[n][C.n_db + i, col]) for n in bases], moduli)
            y = b + sum(int(S_rows[i, v]) * a_pre[v] for v in range(C.n_db))
            noise = OC.centered(y - C.P * delta * int(c.ip_true[col, i]), QP)
            assert abs(noise) < C.P * delta // 8


def test_chain_rescale_is_rounding_by_a_composite_odd_divisor():
    C = OCH.make_chain_params(9, 9, 7, 3, 512, 256)
    P, Q = C.P, C.Q(7)
    rng = np.random.default_rng(3)
    xs = [int(v) for v in rng.integers(0, 2 ** 62, 200)] + [0, P // 2, P // 2 + 1, P - 1, Q * P - 1]
    xs += [int(a) * P + int(b) for a, b in zip(rng.integers(0, 2 ** 40, 50), rng.integers(0, P, 50))]
    for x in xs:
        f = Fraction(x, P)
        assert OCH.rescale(x, P, Q) == (f + Fraction(1, 2)).__floor__() % Q
