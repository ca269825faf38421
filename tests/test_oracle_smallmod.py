"""Pins of the oracle's small-modulus product forms (Section 6.3, fast products with int8
arithmetic) against Python big-integer arithmetic and the paper's printed constants.

* Both forms (RNS over small coprime moduli; M + n M' modulo n^2) give A B mod q equal to the
  big-integer product, on random and extreme entries of a 36-bit prime q.
* The splits reconstruct their input and fit int8.
* The moduli cover the product bound, and one modulus fewer provably does not.
* The paper's counts: simple RNS over prime powers below 2^8 gives 53 moduli and 2^354.83; the
  n^2 form over the primes 127..253 gives 48 int8 planes (its product is 2^360.8, against the
  printed 2^357: a reading recorded in the design notes).
"""
import math

import numpy as np
import pytest

from oracle import smallmod as SM
from oracle.params import ntt_primes

Q = ntt_primes(2)[1]  # a 36-bit prime of the library's basis


def _is_prime(n):
    return n > 1 and all(n % d for d in range(2, math.isqrt(n) + 1))


def _bigint_matmul_mod(A, B, q):
    r, k = A.shape
    c = B.shape[1]
    out = np.empty((r, c), dtype=np.int64)
    for i in range(r):
        for j in range(c):
            out[i, j] = sum(int(A[i, t]) * int(B[t, j]) for t in range(k)) % q
    return out


def _operands(rng, r, k, c, q):
    A = rng.integers(0, q, (r, k), dtype=np.int64)
    B = rng.integers(0, q, (k, c), dtype=np.int64)
    h = (q - 1) // 2
    A[0, :] = h            # extreme centered values: the product bound is reached on row 0 x col 0
    B[:, 0] = h
    A[1, :] = h + 1        # = -h after centering
    A[2, :3] = [0, 1, q - 1]
    return A, B


def test_rns_moduli_are_pairwise_coprime_and_fit_int8():
    ms = SM.RNS_MODULI
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(ms) for b in ms[i + 1:])
    x = np.array([-(2 ** 35), -1, 0, 1, 2 ** 35 - 1, 12345678901, -98765432101], dtype=np.int64)
    for m in ms:
        r = SM.balanced(x, m)
        assert r.min() >= -128 and r.max() <= 127
        assert np.all(np.mod(r - x, m) == 0)


def test_paper_counts_of_the_two_techniques():
    # simple RNS: prime powers p^floor(8 log 2 / log p) < 2^8 over the primes 3 <= p <= 253
    mods = [p ** int(math.floor(8 * math.log(2) / math.log(p))) for p in range(3, 254) if _is_prime(p)]
    assert len(mods) == 53 and max(mods) < 256
    assert abs(sum(math.log2(m) for m in mods) - 354.83) < 0.005
    # the n^2 form: primes 127 <= n <= 253, two int8 planes each
    assert len(SM.P2_BASES) == 24 and 2 * len(SM.P2_BASES) == 48
    assert abs(sum(2 * math.log2(n) for n in SM.P2_BASES) - 360.8) < 0.05


@pytest.mark.parametrize("form", ["rns", "p2"])
def test_small_modulus_product_equals_bigint_product(form):
    rng = np.random.default_rng(5)
    A, B = _operands(rng, 5, 40, 4, Q)
    fn = SM.rns_matmul_mod if form == "rns" else SM.p2_matmul_mod
    assert np.array_equal(fn(A, B, Q), _bigint_matmul_mod(A, B, Q))


def test_moduli_cover_the_bound_and_one_fewer_fails():
    K = 20992
    ms = SM.rns_moduli_for(K, Q)
    assert len(ms) == 11 and math.prod(ms) >= SM.product_bound(K, Q)
    assert math.prod(ms[:-1]) < SM.product_bound(K, Q)
    bs = SM.p2_bases_for(K, Q)
    assert len(bs) == 6 and math.prod(n * n for n in bs) >= SM.product_bound(K, Q)
    # worst case S = K h^2 (all entries h): exact with the chosen moduli, wrong with one fewer
    h = (Q - 1) // 2
    S = K * h * h
    assert SM.crt([S % m for m in ms], ms) == S
    short = ms[:-1]
    assert SM.crt([S % m for m in short], short) != S


def test_splits_reconstruct_and_fit_int8():
    rng = np.random.default_rng(6)
    x = SM.centered(rng.integers(0, Q, 200, dtype=np.int64), Q)
    ms = SM.RNS_MODULI[:11]
    planes = SM.rns_split(x, ms)
    M = math.prod(ms)
    for i in range(len(x)):
        v = SM.crt([int(p[i]) for p in planes], ms)
        assert (v - M if v > M // 2 else v) == int(x[i])
    for n in SM.P2_BASES[:6]:
        a, b = SM.p2_split(x, n)
        assert np.abs(a.astype(int)).max() <= (n - 1) // 2 and np.abs(b.astype(int)).max() <= (n - 1) // 2
        assert np.all(np.mod(a.astype(np.int64) + n * b.astype(np.int64) - x, n * n) == 0)
