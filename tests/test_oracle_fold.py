"""Pins of the normalise-and-fold oracle (oracle/fold.py; Section 4, Algorithm 2, Appendix C.2).

Each step is checked against something other than itself:
  * the encoder (an inverse DFT of length N/2) against the definition of Ecd summed directly, within the
    rounding, and the slot order against evaluation of the polynomial at the complex roots zeta^(5^j)
    (numpy);
  * the automorphism of Rot_r against slot rotation in the direction of Section 4.3 (slot i of
    Rot_r(v) holds v_(i - r)), by evaluation at the roots;
  * the sparse secret's weight and values;
  * key switching by the decryption equation with numpy.polymul products (not oracle.bigmul), the
    same small error modulo every prime;
  * RS, and the relinearised product's single RS by p q_l, by Fraction rounding of the CRT value;
  * products, rotations, f and the whole fold by decryption against the plain values (Appendix C.2's
    polynomial evaluated by numpy.polyval), within bounds derived from the noise.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import fold as F

LOGN = 7


@pytest.fixture(scope="module")
def keys():
    P = F.fold_params(LOGN, 4)
    return F.fold_keygen(P, 11, F.rot_amounts(4, 6))


def _negfold(x, y, q=None):
    """x y mod X^N + 1 by numpy.polymul on Python integers (optionally reduced mod q)."""
    n = len(x)
    full = np.polymul(np.array([int(v) for v in x[::-1]], dtype=object),
                      np.array([int(v) for v in y[::-1]], dtype=object))[::-1]
    full = list(full) + [0] * (2 * n - len(full))
    out = [full[i] - full[i + n] for i in range(n)]
    return [v % q for v in out] if q else out


def _roots_eval(m, log_n):
    """m(zeta^(5^j)) for j < N/2 by numpy.polyval at complex roots."""
    n = 1 << log_n
    g = np.array([pow(5, j, 2 * n) for j in range(n // 2)])
    z = np.exp(1j * np.pi * g / n)
    return np.polyval(np.array([float(v) for v in m[::-1]]), z)


@pytest.mark.parametrize("log_n", [6, 7, 10])
def test_encoder_rounds_the_definition(log_n):
    """Ecd by the length-N/2 inverse DFT against (2/N) sum_j z_j cos(pi i g_j / N) summed directly: within
    1/2 (the rounding) plus the transforms' floating-point error, on both signs and a wide range."""
    n = 1 << log_n
    rng = np.random.default_rng(log_n)
    w = rng.integers(-(1 << 26), 1 << 26, n // 2)
    w[: n // 8] = rng.integers(-3, 4, n // 8)
    e = 6
    m = F.encode(w, log_n, e)
    g = np.array([pow(5, j, 2 * n) for j in range(n // 2)])
    i = np.arange(n)
    exact = (2.0 / n) * (np.cos(np.pi * ((i[:, None] * g[None, :]) % (2 * n)) / n) @ (w * 2.0 ** e))
    assert float(np.max(np.abs(m - exact))) <= 0.5 + 1e-12 * float(np.abs(w).max()) * 2.0 ** e * log_n


def test_slots_are_the_evaluations_at_the_powers_of_5():
    n = 1 << LOGN
    rng = np.random.default_rng(1)
    m = rng.integers(-1000, 1000, n)
    want = _roots_eval(m, LOGN)
    assert np.allclose(F.decode(m, LOGN, 1.0), want.real, atol=1e-8)
    z = rng.integers(-5000, 5000, n // 2)
    back = F.decode(F.encode(z, LOGN, 10), LOGN, 2.0 ** 10)
    assert float(np.max(np.abs(back - z))) < 0.05
    assert np.allclose(_roots_eval(F.encode(z, LOGN, 10), LOGN).imag / 2 ** 10, 0, atol=0.05)


@pytest.mark.parametrize("r", [1, 3, 20])
def test_rotation_automorphism_moves_slot_i_to_i_plus_r(r):
    P = F.fold_params(LOGN, 4)
    rng = np.random.default_rng(r)
    z = rng.integers(-5000, 5000, P.slots)
    m = F.encode(z, LOGN, 10)
    got = _roots_eval(F.automorphism(m, F.rot_galois(P, r)), LOGN).real / 2 ** 10
    assert float(np.max(np.abs(got - np.roll(z, r)))) < 0.05


def test_sparse_secret_weight_and_values():
    s = F.sparse_secret(3, 1 << 10)
    assert int(np.count_nonzero(s)) == F.H_WEIGHT and set(np.unique(s[s != 0])) <= {-1, 1}
    assert not np.array_equal(s, F.sparse_secret(4, 1 << 10))
    assert np.array_equal(s, F.sparse_secret(3, 1 << 10))


def _ks_error(FK, level, x, s_from, key):
    P = FK.P
    B, A = F.key_switch(P, level, x, key)
    errs = []
    for z in P.moduli(level):
        lhs = [(int(b) + v) % z for b, v in zip(B[z], _negfold(A[z], FK.s, z))]
        rhs = _negfold(x[z], s_from, z)
        errs.append([F.centered(u - v, z) for u, v in zip(lhs, rhs)])
    return errs


@pytest.mark.parametrize("level,rotation", [(1, True), (1, False), (3, False)])
def test_key_switch_satisfies_the_decryption_equation(keys, level, rotation):
    P = keys.P
    rng = np.random.default_rng(level)
    x = {z: rng.integers(0, z, P.n) for z in P.moduli(level)}
    if rotation:
        sg = F.automorphism(keys.s, F.rot_galois(P, 3))
        errs = _ks_error(keys, level, x, [int(v) for v in sg], keys.rot[3])
    else:
        errs = _ks_error(keys, level, x, _negfold(keys.s, keys.s), keys.relin[level])
    for e in errs[1:]:
        assert e == errs[0]                      # one integer error, the same modulo every prime
    qmax = max(P.moduli(level))
    bound = (level + 1) * P.n * 19 * qmax // P.p + F.H_WEIGHT + 2
    assert max(abs(v) for v in errs[0]) <= bound


def test_rescale_rounds_to_nearest(keys):
    P = keys.P
    rng = np.random.default_rng(5)
    primes = P.moduli(3)
    res = {z: rng.integers(0, z, 16) for z in primes}
    out = F.rescale_by(res, primes[-1], primes[:-1])
    Q = P.Q(3)
    for t in range(16):
        x = 0
        for z in primes:
            Mi = Q // z
            x += int(res[z][t]) * Mi * pow(Mi, -1, z)
        x = F.centered(x, Q)
        want = Fraction(x, primes[-1])
        rounded = int(want + Fraction(1, 2)) if want >= 0 else -int(-want + Fraction(1, 2))
        if abs(want - int(want)) == Fraction(1, 2):
            continue
        for z in primes[:-1]:
            assert int(out[z][t]) == rounded % z


def test_rescale_by_p_q_rounds_to_nearest(keys):
    """RS_{p q_l} of a relinearised product (one division by the composite p q_3) against Fraction rounding
    of the CRT value over q_0 .. q_3 and p."""
    P = keys.P
    rng = np.random.default_rng(6)
    primes = P.moduli(3)
    mods = primes + [P.p]
    res = {z: rng.integers(0, z, 16) for z in mods}
    out = F.rescale_by_two(res, P.p, primes[-1], primes[:-1])
    M = 1
    for z in mods:
        M *= z
    D = P.p * primes[-1]
    for t in range(16):
        x = 0
        for z in mods:
            Mi = M // z
            x += int(res[z][t]) * Mi * pow(Mi, -1, z)
        x = F.centered(x, M)
        want = Fraction(x, D)
        rounded = int(want + Fraction(1, 2)) if want >= 0 else -int(-want + Fraction(1, 2))
        if abs(want - int(want)) == Fraction(1, 2):
            continue
        for z in primes[:-1]:
            assert int(out[z][t]) == rounded % z


def _inputs(P, n, seed):
    rng = np.random.default_rng(seed)
    counts = rng.integers(800, 1200, (n, P.slots))
    scores = np.clip(rng.normal(0.008, 0.06, (n, P.slots)), -0.3, 0.3)
    scores[0, 2] = 0.45
    scores[n - 1, 5] = 0.52
    return np.rint(scores * counts).astype(np.int64), counts


def test_products_rotations_and_f_decrypt_to_the_plain_values(keys):
    P = keys.P
    S = F.schedule(P)
    ip, counts = _inputs(P, 2, 7)
    cts = [F.encrypt(keys, ip[i], 13, i) for i in range(2)]
    assert float(np.max(np.abs(F.decode(F.decrypt(keys, cts[0]), LOGN, 2.0 ** F.LOG_IN) - ip[0]))) < 0.5
    x = [F.normalise(keys, c, cn) for c, cn in zip(cts, counts)]
    xv = [ip[i] / counts[i] for i in range(2)]
    for i in range(2):
        assert float(np.max(np.abs(F.decode(F.decrypt(keys, x[i]), LOGN, S.S1) - xv[i]))) < 1e-4
    prod = F.mul(keys, x[0], x[1])
    assert float(np.max(np.abs(F.decode(F.decrypt(keys, prod), LOGN, S.S2) - xv[0] * xv[1]))) < 1e-4
    y = F.poly_f(keys, x[0])
    assert y[0] == 1
    fx = F.f_plain(xv[0])
    assert float(np.max(np.abs(F.decode(F.decrypt(keys, y), LOGN, S.G) - fx))) < 5e-3
    ry = F.rotate(keys, y, 3)
    assert float(np.max(np.abs(F.decode(F.decrypt(keys, ry), LOGN, S.G) - np.roll(fx, 3)))) < 5e-3


def test_schedule_joins_terms_at_equal_scales():
    P = F.fold_params(LOGN)
    S = F.schedule(P)
    q = [float(v) for v in P.q]
    assert S.G == S.F * q[1]                              # f at level 1 becomes F after RS by q_1
    assert S.S4 * S.U == pytest.approx(S.G, rel=1e-14)
    assert S.S2 * S.T3 / q[2] == pytest.approx(S.U, rel=1e-14)
    assert S.S2 * S.T1 / q[2] == pytest.approx(S.G, rel=1e-14)
    # the integer constants carry c_j at their scales to 2^-20
    E = [S.G, S.G * q[3] / S.S1, S.T1, S.T1 * q[3] / S.S1, S.U, S.U * q[3] / S.S1, S.T3, S.T3 * q[3] / S.S1]
    for kj, cj, ej in zip(S.k, F.COEFFS, E):
        assert abs(kj / ej - cj) <= 2.0 ** -20 * max(1.0, abs(cj))


@pytest.mark.parametrize("rho", [6, 4])
def test_fold_decrypts_to_the_rotated_sum_of_f(keys, rho):
    P = keys.P
    n = 2 * rho if rho == 4 else rho
    ip, counts = _inputs(P, n, rho)
    cts = [F.encrypt(keys, ip[i], 17, i) for i in range(n)]
    out = F.fold(keys, cts, counts, rho)
    want = F.fold_plain(ip, counts, rho, P.k)
    assert len(out) == len(want) == (n // rho) * -(-rho // P.k)
    S = F.schedule(P)
    for o, wv in zip(out, want):
        assert o[0] == 0
        got = F.decode(F.decrypt(keys, o), LOGN, S.F)
        assert float(np.max(np.abs(got - wv))) < 0.01
