"""Pins of the FormatSwitch oracle (oracle/formatswitch.py, Appendix C.1) and of its exact large-degree
product (oracle/bigmul.py).

The product is pinned against the Neg(s)-matrix definition at small degrees, against the definition sum
on sampled coefficients at degree 2^16, and by monomials.  Every FormatSwitch step is pinned by the
decryption equation it must satisfy, with the secret products taken by numpy.polymul folded mod
X^n + 1 (independent of bigmul): the transmission ciphertexts under s_T, the key switch
(B + A s' (X^rho) = a s_T + small), the ring switch under s', the MSRLWE conversion under every s_j,
the final query under the CCMM secrets at the CCMM's scale; and end to end, a CCMM of the switched
query against an encrypted database decrypts to the popcount inner products.
"""
import numpy as np
import pytest

from oracle import bigmul as B
from oracle import ckks as OC
from oracle import formatswitch as FS
from oracle import iris as OI
from oracle import params as OP
from oracle import ring as R

Q36 = OP.ntt_primes(1)[0]


def _fold(s, a, q):
    """s * a mod (X^n + 1, q) by numpy.polymul on Python integers."""
    n = len(s)
    full = np.polymul(np.array([int(x) for x in s[::-1]], dtype=object),
                      np.array([int(x) for x in a[::-1]], dtype=object))[::-1]
    out = [0] * n
    for i, v in enumerate(full):
        if i < n:
            out[i] += v
        else:
            out[i - n] -= v
    return np.array([v % q for v in out], dtype=object)


def _err(x, q):
    return max(abs(OC.centered(int(v), q)) for v in x)


@pytest.mark.parametrize("n", [2, 16, 512])
def test_bigmul_equals_the_neg_matrix_product(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, Q36, n)
    s = rng.integers(-1, 2, n)
    want = (R.neg_matrix(s).astype(object).dot(a.astype(object))) % Q36
    assert np.array_equal(B.negmul_small(s, a, Q36).astype(object), want)
    b = rng.integers(0, Q36, n)
    assert np.array_equal(B.negmul_mod(b, a, Q36).astype(object), _fold(b, a, Q36))


def test_bigmul_at_degree_2_16_by_definition_and_monomials():
    n = 1 << 16
    rng = np.random.default_rng(7)
    a, b = rng.integers(0, Q36, n), rng.integers(0, Q36, n)
    got = B.negmul_mod(a, b, Q36)
    for t in (0, 1, 4097, 30000, n - 1):
        v = sum(int(a[u]) * int(b[t - u]) for u in range(t + 1)) - sum(int(a[u]) * int(b[t - u + n]) for u in range(t + 1, n))
        assert int(got[t]) == v % Q36
    x = np.zeros(n, dtype=np.int64)
    x[n - 3] = 1                                             # X^(n-3) X^5 = -X^2
    y = np.zeros(n, dtype=np.int64)
    y[5] = 1
    z = B.negmul_mod(x, y, Q36)
    assert int(z[2]) == Q36 - 1 and int(np.count_nonzero(z)) == 1


@pytest.fixture(scope="module")
def fs():
    # ring degrees 2^10 -> 2^7 (rho 8), d2 = 200 (two chunks), level 1 (transmission at two primes)
    P = OP.make_params(7, 7, 2, 200, 64)
    F = FS.fs_keygen(P, 1, 10, 5)
    rng = np.random.default_rng(0)
    codes = rng.integers(0, 2, (2, 200)).astype(np.uint8)
    masks = (rng.random((2, 200)) < 0.9).astype(np.uint8)
    qc, qm = OI.shifted_queries(codes, masks, np.array([0, 3]))
    m = OI.ternary(qc, qm)
    ct = FS.encrypt_transmit(F, m, 9)
    return P, F, m, ct, codes, masks, qc, qm


def test_transmission_ciphertexts_decrypt_under_s_T(fs):
    P, F, m, ct, *_ = fs
    scale = P.delta(1) * P.q[1]
    for q in F.primes_in():
        for col in range(m.shape[0] * P.k):
            c, j = divmod(col, P.k)
            mt = np.zeros(F.n_t, dtype=np.int64)
            lo, hi = j * P.n_q, min((j + 1) * P.n_q, P.d2)
            mt[:(hi - lo) * F.rho:F.rho] = m[c, lo:hi]
            a, b = ct[q][col]
            assert _err((b + _fold(F.s_t, a, q) - scale * mt) % q, q) <= 19


def test_key_switch_moves_a_to_the_embedded_secret(fs):
    P, F, m, ct, *_ = fs
    primes = F.primes_in()
    a = {q: ct[q][0, 0] for q in primes}
    A, Bk = FS.key_switch(F, a, lambda z, i: F.rk[z][i])
    s_emb = FS._embed(F.s_r, F.rho)
    for q in primes:
        e = (Bk[q] + _fold(s_emb, A[q], q) - _fold(F.s_t, a[q], q)) % q
        assert _err(e, q) < 1 << 12               # sum_i d_i e_i / p plus the rounding terms


def test_ring_switch_and_conversion_decrypt_under_their_secrets(fs):
    P, F, m, ct, *_ = fs
    primes = F.primes_in()
    scale = P.delta(1) * P.q[1]
    chunks = [FS.ring_switch(F, ct, j) for j in range(P.k)]
    for j, (a1, b1) in enumerate(chunks):
        lo, hi = j * P.n_q, min((j + 1) * P.n_q, P.d2)
        mj = np.zeros(P.n_q, dtype=np.int64)
        mj[:hi - lo] = m[0, lo:hi]
        for q in primes:
            assert _err((b1[q] + _fold(F.s_r, a1[q], q) - scale * mj) % q, q) < 1 << 12
    a, bs = FS.convert(F, chunks)
    for j in range(P.k):
        lo, hi = j * P.n_q, min((j + 1) * P.n_q, P.d2)
        mj = np.zeros(P.n_q, dtype=np.int64)
        mj[:hi - lo] = m[0, lo:hi]
        for q in primes:
            assert _err((bs[j][q] + _fold(F.keys.s[j], a[q], q) - scale * mj) % q, q) < 1 << 13


def test_switched_query_decrypts_at_the_ccmm_scale_and_the_ccmm_gives_the_popcounts(fs):
    P, F, m, ct, codes, masks, qc, qm = fs
    XT = FS.format_switch(F, ct, m.shape[0])
    q, delta = P.q[0], P.delta(1)
    for c in range(m.shape[0]):
        b, a = XT[0][c, :P.d2], XT[0][c, P.d2:]
        for j in range(P.k):
            lo, hi = j * P.n_q, min((j + 1) * P.n_q, P.d2)
            sa = _fold(F.keys.s[j], a, q)
            e = [(int(b[t]) + int(sa[t - lo]) - delta * int(m[c, t])) for t in range(lo, hi)]
            assert _err(e, q) <= 64                       # the modulus switch divides the noise by q_1
    rng = np.random.default_rng(1)
    db_codes = rng.integers(0, 2, (64, P.d2)).astype(np.uint8)
    db_masks = (rng.random((64, P.d2)) < 0.9).astype(np.uint8)
    db_codes[5] = codes[0]
    db_masks[5] = masks[0]
    D = OC.encrypt_db(F.keys, OI.ternary(db_codes, db_masks), 3)
    out = OC.ccmm(P, D, XT, 1, 0, 64)
    _, ip = OC.decrypt(F.keys, out, 1, 0, 64)
    ip_true, _ = OI.truth(qc, qm, db_codes, db_masks)
    assert np.array_equal(ip, ip_true)
