"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something other than its own formulas:
library routines that compute the same object (numpy's Philox, numpy.polymul),
brute force on tiny inputs, a hand-worked example (tests/golden), closed forms,
and the masked-Hamming identity of Section 2.1.3 evaluated by popcount.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import hfe_synth as S
from oracle import ckks as OC
from oracle import iris as OI
from oracle import params as OP
from oracle import prng
from oracle import ring as OR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ primes

def _trial_division_prime(n: int) -> bool:
    r = math.isqrt(n)
    cand = np.arange(2, r + 1, dtype=np.int64)
    return n > 1 and not np.any(n % cand == 0)


def test_primes_are_prime_by_trial_division_and_maximal():
    ps = OP.ntt_primes(6)
    step = 1 << 17
    for q in ps:
        assert q < (1 << 36) and q % step == 1
        assert _trial_division_prime(q)
    # nothing skipped: every candidate = 1 mod 2^17 between 2^36 and the last prime is composite
    c = ((1 << 36) - 1) // step * step + 1
    found = []
    while c >= ps[-1]:
        if _trial_division_prime(c):
            found.append(c)
        c -= step
    assert found == ps


def test_miller_rabin_matches_trial_division_on_small_range():
    for n in range(2, 5000):
        assert OP.is_prime(n) == _trial_division_prime(n)


def test_delta_is_power_of_two_gap_below_Q():
    P = OP.make_params(14, 13, 3, 12800, 14336)
    for lvl in (1, 2, 3):
        Q = P.Q(lvl)
        d = P.delta(lvl)
        assert d & (d - 1) == 0
        assert d * (1 << 20) <= Q < d * (1 << 21)


# ------------------------------------------------------------------ PRNG

@pytest.mark.parametrize("key", [(0, 0), (1, 2), (260117561, (3 << 32) | 16), (2**64 - 1, 2**63 + 5)])
def test_philox_matches_numpy_philox(key):
    rng = np.random.default_rng(5)
    for _ in range(5):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4)]
        ctr[0] += 1                                  # numpy pre-increments its counter
        ref = np.random.Philox(key=list(key), counter=[ctr[0] - 1] + ctr[1:]).random_raw(4)
        got = prng.philox4x64_10(key[0], key[1], ctr[0], ctr[1], ctr[2], ctr[3])
        assert [int(g) for g in got] == [int(r) for r in ref]


def test_philox_vectorised_matches_scalar():
    c0 = np.arange(17, dtype=np.uint64)
    vec = prng.philox4x64_10(9, 10, c0, 3, 0, 0)
    for i in range(17):
        one = prng.philox4x64_10(9, 10, i, 3, 0, 0)
        assert [int(v[i]) for v in vec] == [int(x) for x in one]


def test_uniform_matrix_equals_elementwise_definition():
    q = OP.ntt_primes(1)[0]
    A = prng.uniform_matrix(7, prng.DBA, 16, 37, 11, q)
    r, c = np.meshgrid(np.arange(37), np.arange(11), indexing="ij")
    B = prng.uniform_mod(7, prng.DBA, 16, r.astype(np.uint64), c.astype(np.uint64), q)
    assert np.array_equal(A, B)
    assert A.min() >= 0 and A.max() < q


def test_uniform_rejection_path_follows_spec():
    q = (1 << 63) + 25                               # bound = q: about half the words are rejected
    idx = np.arange(64, dtype=np.uint64)
    got = prng.uniform_mod(3, 9, 1, idx, np.zeros_like(idx), q)
    for i in range(64):
        w = int(prng.philox4x64_10(3, (9 << 32) | 1, i >> 2, 0, 0, 0)[i & 3])
        if w < q:
            assert got[i] == w % q
        else:
            a = 1
            while True:
                ys = [int(y) for y in prng.philox4x64_10(3, (9 << 32) | 1, i, 0, a, 0)]
                acc = [y for y in ys if y < q]
                if acc:
                    assert got[i] == acc[0] % q
                    break
                a += 1


def test_ternary_frequencies():
    s = prng.ternary(11, prng.QSEC, 0, 30000)
    counts = np.array([(s == v).sum() for v in (-1, 0, 1)])
    chi2 = ((counts - 10000) ** 2 / 10000).sum()
    assert chi2 < 13.8                               # p = 0.001, 2 dof


def test_cdt_table_exact_at_higher_precision_and_close_to_float():
    t80 = prng.cdt_table(80)
    t120 = prng.cdt_table(120)
    assert t80 == t120
    sig2 = 3.2 ** 2
    rho = [math.exp(-x * x / (2 * sig2)) for x in range(20)]
    z = rho[0] + 2 * sum(rho[1:])
    cum = rho[0]
    for j in range(19):
        if j:
            cum += 2 * rho[j]
        assert abs(t80[j] / 2.0**64 - cum / z) < 1e-12
    assert all(a < b for a, b in zip(t80, t80[1:])) and t80[-1] < 2**64


def test_gaussian_distribution_and_matrix_agreement():
    E = prng.gaussian_matrix(5, prng.DBE, 0, 301, 400)
    r, c = np.meshgrid(np.arange(301), np.arange(400), indexing="ij")
    assert np.array_equal(E, prng.gaussian(5, prng.DBE, 0, r.astype(np.uint64), c.astype(np.uint64)))
    pmf = prng.gaussian_pmf()
    n = E.size
    mags = np.abs(E).ravel()
    chi2 = 0.0
    dof = 0
    for j in range(8):
        exp = float(pmf[j]) * n
        chi2 += (int((mags == j).sum()) - exp) ** 2 / exp
        dof += 1
    assert chi2 < 26.1                               # p = 0.001, 7 dof
    assert abs(E.std() - 3.2) < 0.05 and np.abs(E).max() <= 19
    assert abs((E > 0).sum() - (E < 0).sum()) < 4 * math.sqrt(n)


# ------------------------------------------------------------------ ring

def test_neg_matrix_equals_schoolbook_loops():
    rng = np.random.default_rng(1)
    for n in (1, 2, 4, 8, 16):
        s = rng.integers(-1, 2, n)
        a = rng.integers(-1000, 1000, n)
        assert list(OR.neg_matrix(s) @ a) == OR.negmul_schoolbook(list(s), list(a))


def test_negacyclic_monomials():
    n = 8
    for i in range(n):
        for j in range(n):
            xi = np.zeros(n, dtype=np.int64)
            xi[i] = 1
            xj = np.zeros(n, dtype=np.int64)
            xj[j] = 1
            prod = OR.neg_matrix(xi) @ xj
            exp = np.zeros(n, dtype=np.int64)
            exp[(i + j) % n] = 1 if i + j < n else -1
            assert np.array_equal(prod, exp)


def _polymul_fold(s, a):
    n = len(s)
    full = np.polymul(np.asarray(s, dtype=object)[::-1], np.asarray(a, dtype=object)[::-1])[::-1]
    full = list(full) + [0] * (2 * n - len(full))
    return [int(full[t]) - int(full[t + n]) for t in range(n)]


def test_neg_matrix_matches_numpy_polymul_reduced_mod_xn_plus_1():
    rng = np.random.default_rng(2)
    for n in (16, 64, 256):
        s = rng.integers(-1, 2, n)
        a = rng.integers(0, 2**36, n)
        assert list(OR.neg_matrix(s) @ a) == _polymul_fold(s, a)


def test_imatmul_and_modmatmul_against_python_ints():
    rng = np.random.default_rng(3)
    A = rng.integers(0, 2**36, (7, 13))
    A[0, :] = 2**36 - 1
    B = rng.integers(0, 2**36, (13, 5))
    B[:, 0] = 2**36 - 1
    q = OP.ntt_primes(1)[0]
    got = OR.modmatmul(A, B, q)
    for i in range(7):
        for j in range(5):
            assert got[i, j] == sum(int(A[i, k]) * int(B[k, j]) for k in range(13)) % q
    C = rng.integers(-1, 2, (70, 90))
    D = rng.integers(-2**40, 2**40, (90, 66))
    got = OR.imatmul(C, D)
    assert all(got[i, j] == sum(int(C[i, k]) * int(D[k, j]) for k in range(90))
               for i in range(0, 70, 9) for j in range(0, 66, 7))
    with pytest.raises(AssertionError):
        OR.imatmul(np.full((2, 3), 2**40), np.full((3, 2), 2**30))


# ------------------------------------------------------------------ masked Hamming (Section 2.1)

def test_masked_bitvector_identity_and_truth_by_brute_force():
    rng = np.random.default_rng(4)
    c1, m1 = rng.integers(0, 2, (6, 131)), (rng.random((6, 131)) < 0.9).astype(np.uint8)
    c2, m2 = rng.integers(0, 2, (9, 131)), (rng.random((9, 131)) < 0.9).astype(np.uint8)
    ip, ov = OI.truth(c1.astype(np.uint8), m1, c2.astype(np.uint8), m2)
    t1, t2 = OI.ternary(c1, m1).astype(int), OI.ternary(c2, m2).astype(int)
    for a in range(6):
        for b in range(9):
            both = [int(m1[a, t] and m2[b, t]) for t in range(131)]
            hd = sum(int(c1[a, t] != c2[b, t]) * both[t] for t in range(131))
            inner = sum(t1[a, t] * t2[b, t] for t in range(131))
            assert 2 * hd == sum(both) - inner                  # Section 2.1.3 identity
            assert ip[a, b] == inner and ov[a, b] == sum(both)


def test_decision_threshold_semantics():
    ov = np.array([[8, 8, 8, 0]])
    ip = np.array([[2, 3, 1, 5]])                             # score 1/4 is not > 1/4
    assert OI.decide(ip, ov).tolist() == [[False, True, False, False]]


def test_match_per_eye_by_brute_force():
    """match_per_eye: eye e matches iff some decision of its shift columns e * n_shifts + s (the
    eye-major order of shifted_queries) against some database row is true; checked by loops over
    eyes, shifts and rows, on random decisions and on single planted decisions at every position
    (an eye-major / shift-major mix-up or a dropped row fails the single-decision cases)."""
    rng = np.random.default_rng(4)
    n_eyes, n_shifts, rows = 5, 3, 7

    def brute(dec):
        return np.array([any(dec[e * n_shifts + s, r] for s in range(n_shifts) for r in range(rows))
                         for e in range(n_eyes)])

    for _ in range(20):
        dec = rng.random((n_eyes * n_shifts, rows)) < 0.03
        assert np.array_equal(OI.match_per_eye(dec, n_shifts), brute(dec))
    for col in range(n_eyes * n_shifts):
        for r in range(rows):
            dec = np.zeros((n_eyes * n_shifts, rows), dtype=bool)
            dec[col, r] = True
            want = np.zeros(n_eyes, dtype=bool)
            want[col // n_shifts] = True
            assert np.array_equal(OI.match_per_eye(dec, n_shifts), want)
    qc = np.zeros((2, 8), dtype=np.uint8)
    qm = np.ones((2, 8), dtype=np.uint8)
    qc[1, 0] = 1                                            # eye 1 differs from eye 0 at bit 0
    cols_c, _ = OI.shifted_queries(qc, qm, np.array([0, 1, 2]))
    assert cols_c[3:].any() and not cols_c[:3].any()        # columns 3..5 are eye 1's shifts


def test_shifted_queries_roll_code_and_mask_together():
    c = np.array([[1, 0, 0, 0, 0]], dtype=np.uint8)
    m = np.array([[1, 1, 0, 0, 0]], dtype=np.uint8)
    qc, qm = OI.shifted_queries(c, m, np.array([-1, 0, 2]))
    assert qc.tolist() == [[0, 0, 0, 0, 1], [1, 0, 0, 0, 0], [0, 0, 1, 0, 0]]
    assert qm.tolist() == [[1, 0, 0, 0, 1], [1, 1, 0, 0, 0], [0, 0, 1, 1, 0]]


# ------------------------------------------------------------------ rescale (Section 2.2.4)

def test_rescale_matches_fraction_rounding_and_centered_residue_form():
    rng = np.random.default_rng(6)
    p = OP.ntt_primes(1)[0]
    Q = 1
    for qi in OP.ntt_primes(4)[1:]:
        Q *= qi
    for _ in range(300):
        x = int(rng.integers(0, 2**62)) * int(rng.integers(0, 2**62)) % (Q * p)
        exp = math.floor(Fraction(x, p) + Fraction(1, 2)) % Q
        assert OC.rescale_p(x, p, Q) == exp
        assert (x - OC.centered(x, p)) // p % Q == exp


# ------------------------------------------------------------------ hand-worked CCMM

def test_golden_worked_example_ring_degree_2():
    g = json.load(open(os.path.join(GOLDEN, "worked_n2.json")))
    P = OP.Params(log_n_db=1, log_n_q=1, q=tuple(g["params"]["q"]), p=g["params"]["p"],
                  d2=2, max_db_rows=2, gap=g["params"]["gap"])
    assert P.delta(1) == g["params"]["delta"]
    keys = OC.Keys(P, 0, np.array([g["s_q"]]), np.array([g["s_db"]]))
    SQ = OC.s_q_matrix(keys)
    SDB = OC.s_db_rows(keys, range(2))
    assert SQ.tolist() == [[1, 1], [-1, 1]] and SDB.tolist() == [[0, -1], [1, 0]]
    m_db = np.array(g["m_db"])
    XT = OC.encrypt_query_with(P, SQ, np.array(g["m_q_rows"]), 1,
                               {0: np.array(g["query_a"]).reshape(2, 1)},
                               np.array(g["query_e"]).reshape(2, 1))
    assert XT[0][0].tolist() == g["expect"]["xt_q0"]
    D = OC.encrypt_db_with(P, SQ, SDB, m_db,
                           {0: np.array(g["db_a"]["q0"]), prng.P_ID: np.array(g["db_a"]["p"])},
                           np.array(g["db_e"]))
    assert D[0].tolist() == g["expect"]["d_q0"] and D[prng.P_ID].tolist() == g["expect"]["d_p"]
    C = OC.ccmm_pre_rescale(P, D, XT, 1, 0, 2)
    assert C[0][:, 0].tolist() == g["expect"]["c_q0"] and C[prng.P_ID][:, 0].tolist() == g["expect"]["c_p"]
    out = OC.ccmm(P, D, XT, 1, 0, 2)
    assert out[0][0].tolist() == g["expect"]["out_q0"]
    v, ip = OC.decrypt(keys, out, 1, 0, 2)
    assert [int(x * 8) for x in v[0]] == g["expect"]["y"] and ip[0].tolist() == g["expect"]["ip"]
