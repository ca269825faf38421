"""Normalise and fold: the loop body of Algorithm 2 after the CCMM (oracle).

Test infrastructure: only the tests, the package's smoke check and the benchmark's CPU baseline use it.

What is computed (Section 4.1-4.3, Algorithm 2, Appendix C.2).  A block of rho score ciphertexts
ct_c (c < rho, one query column c against N/2 database entries in the slots) becomes ceil(rho / k)
folded ciphertexts

    ct'_r = sum_{r' < min(k, rho - r k)} Rot_{r k + r'}( f( ct_{r k + r'} (.) mu_{r k + r'} ) )

where mu_c = Ecd(1 / ||m_q,c AND m_db,j||_1 over the slots j) normalises the inner products into scores
(a plaintext-ciphertext product), f is the degree-7 folding polynomial of Appendix C.2 (k = 16), and
Rot_r moves slot i to slot i + r, so that slot i of Rot_r(v) holds the score of database entry i - r
(Section 4.3).  Everything is CKKS in coefficient form here: a ciphertext at level l is (b, a) with
residues mod q_0 .. q_l, and b + a s = Delta m + e.

Parameters (the paper fixes degree, depth, scale and key weight; the rest are readings):
  ring degree N = 2^log_n, N/2 real slots; slot j is the evaluation at zeta^(5^j mod 2N), zeta = e^(i pi / N)
  q_0 a 36-bit prime (holds the folded sum), q_1 .. q_3 primes near 2^23 (the three levels of f at
  Delta = 2^23, Appendix C.2), q_4 a 36-bit prime (the normalisation's level), p a 36-bit special prime
  for key switching; all = 1 mod 2^17
  secret s ternary of Hamming weight h = 32 (Appendix C.2)
  input: the inner products IP (integers) at scale 2^20 at level 4; mu encoded at scale 2^40
  normalise: x = RS_{q_4}(ct (.) Ecd(mu)) at level 3, scale S1 = 2^60 / q_4 (about 2^24)
  f = (c0 + c1 x) + x^2 (c2 + c3 x) + x^4 ((c4 + c5 x) + x^2 (c6 + c7 x)): three levels, five products
  with relinearisation; every constant is encoded at the scale that makes the terms it joins equal in
  scale, so that f sits at level 1 with scale G = 2^24 q_1 (up to the constants' rounding); the last
  rescale waits until the rotations and the sum of a group are done (rotations at level 1, where the
  key-switching error is far below the scale), and brings the folded sum to level 0, scale F = 2^24
  Rot_{r k + r'} = Rot_{r k} o Rot_{r'}: the k - 1 rotations inside a group, then one by r k on the sum
  key switching: one digit per prime, d_i = [a (Q_l / q_i)^-1]_{q_i}, keys
  K_i = (k_i, -k_i s + p (Q_l / q_i) s_from + e_i) mod Q_l p, then RS_p (as for FormatSwitch); a product
  that is rescaled divides p (d0, d1) + sum_i d_i K_i by p q_l in one rounding (RS_{p q_l}) instead of
  RS_p and then RS_{q_l}

Encoding.  Ecd rounds the real polynomial whose slots are the given values, (2/N) sum_j z_j
cos(pi i g_j / N) with g_j = 5^j mod 2N, to integers.  It is computed as a length-N/2 inverse DFT
(encode below) in a fixed sequence of IEEE double operations, so that another implementation of the
same sequence takes the same rounding decisions; it is pinned against the definition.  The decoder is
the floating-point definition (tests only).

Random streams (Philox, the layout of oracle.prng):
  FSEC  sub 0: word t orders the coefficients, the h smallest carry the secret's non-zeros; sub 1: sign
  FKA   sub = stream id of the slot's prime: key masks at (coef t, key kappa * 8 + digit i)
  FKE   sub 0: key errors at (coef t, kappa * 8 + i)
  FXA   sub = stream id: input ciphertext masks at (coef t, ciphertext index)
  FXE   sub 0: input errors at (coef t, ciphertext index)
  key kappa: relinearisation at level l is l - 1 (l = 1, 2, 3); rotation by the a-th amount (level 1) is
  3 + a.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import prng
from .bigmul import negmul_mod
from .ckks import centered
from .params import ntt_primes

FSEC, FKA, FKE, FXA, FXE = 15, 16, 17, 18, 19
H_WEIGHT = 32
# f(x) = sum_j c_j x^j, the folding polynomial of Appendix C.2 (degree 7, k = 16)
COEFFS = (0.004105, -0.173510, -2.528271, 24.347349, 124.161550, -412.746212, 376.961251, 106.553952)
LOG_IN = 20          # scale of the input inner products
LOG_MU = 40          # scale of the normalisation plaintext
LOG_F = 24           # scale of the folded result
W_BITS = 30          # mu_j is encoded from w_j = round(2^30 / count_j)
LEVELS = 4           # q_1 .. q_4: three levels of f + normalise
ROT_LEVEL = 1        # level of the rotations and group sums


@dataclasses.dataclass(frozen=True)
class FoldParams:
    log_n: int
    q: Tuple[int, ...]       # q_0 .. q_4
    p: int
    k: int                   # folding factor

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def slots(self) -> int:
        return self.n // 2

    def sid(self, z: int) -> int:
        """Random-stream id of modulus z: i for q_i, 16 for p."""
        return prng.P_ID if z == self.p else self.q.index(z)

    def moduli(self, level: int) -> List[int]:
        return list(self.q[: level + 1])

    def Q(self, level: int) -> int:
        out = 1
        for z in self.q[: level + 1]:
            out *= z
        return out


def fold_params(log_n: int, k: int = 16) -> FoldParams:
    big = ntt_primes(3)                       # 36-bit, = 1 mod 2^17: q_0, p, q_4
    small = ntt_primes(3, 23, 17)             # the three largest below 2^23: q_1 .. q_3
    return FoldParams(log_n, (big[0],) + tuple(small) + (big[2],), big[1], k)


# ---------------------------------------------------------------- encoding

def galois_5(n: int) -> np.ndarray:
    """g_j = 5^j mod 2N for j < N/2."""
    out = np.empty(n // 2, dtype=np.int64)
    g = 1
    for j in range(n // 2):
        out[j] = g
        g = g * 5 % (2 * n)
    return out


def _brv(x: int, bits: int) -> int:
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def slot_tables(log_n: int):
    """W[u] = e^(-2 pi i u / M) (u < M/2), Z[i] = zeta^i (i < M), pos[j] = brv(k_j), k_j = (g_j - 1) / 4,
    M = N/2; cosines and sines from the C library (math.cos, math.sin)."""
    n = 1 << log_n
    m = n // 2
    W = np.array([[math.cos(2.0 * math.pi * u / m), -math.sin(2.0 * math.pi * u / m)] for u in range(m // 2)])
    Z = np.array([[math.cos(math.pi * i / n), math.sin(math.pi * i / n)] for i in range(m)])
    k = (galois_5(n) - 1) // 4
    pos = np.array([_brv(int(v), log_n - 1) for v in k], dtype=np.int64)
    return W.reshape(-1, 2), Z, pos, k


def encode(w: np.ndarray, log_n: int, e: int) -> np.ndarray:
    """Integer slot values w (N/2 of them) at scale 2^e -> plaintext coefficients (int64, N).

    The real polynomial m with m(zeta^(g_j)) = w_j 2^e: with M = N/2, g_j = 1 + 4 k_j and
    u_i = m_i + i m_(i+M), the slots are the DFT of length M (root w = e^(2 pi i / M)) of u_i zeta^i at
    k_j, so u_i = zeta^-i (1/M) sum_k zhat_k w^(-i k).  The inverse DFT is the radix-2 transform in
    decimation in time on bit-reversed input, each butterfly (a, c) -> (a + W c, a - W c) with
    W c = (Wr cr - Wi ci, Wr ci + Wi cr), in IEEE doubles (numpy's elementwise products and sums, no
    fused multiply-add); then u_i = ((xr c + xi s) / M, (xi c - xr s) / M) with zeta^i = (c, s), and
    m_i = floor(Re u_i + 1/2), m_(i+M) = floor(Im u_i + 1/2)."""
    n = 1 << log_n
    M = n // 2
    W, Z, pos, _ = slot_tables(log_n)
    w = np.asarray(w, dtype=np.int64)
    assert w.shape == (M,) and int(np.max(np.abs(w), initial=0)) < (1 << 52 - max(e, 0))
    xr = np.zeros(M)
    xi = np.zeros(M)
    xr[pos] = w.astype(np.float64) * float(2.0 ** e)
    half = 1
    while half < M:
        step = M // (2 * half)
        b = np.arange(M // 2)
        t = b % half
        ia = (b // half) * 2 * half + t
        ic = ia + half
        wr, wi = W[t * step, 0], W[t * step, 1]
        cr, ci = xr[ic], xi[ic]
        pr = wr * cr - wi * ci
        pi = wr * ci + wi * cr
        ar, ai = xr[ia].copy(), xi[ia].copy()
        xr[ia], xi[ia] = ar + pr, ai + pi
        xr[ic], xi[ic] = ar - pr, ai - pi
        half *= 2
    inv_m = 1.0 / M
    c, s_ = Z[:, 0], Z[:, 1]
    ur = (xr * c + xi * s_) * inv_m
    ui = (xi * c - xr * s_) * inv_m
    return np.concatenate([np.floor(ur + 0.5), np.floor(ui + 0.5)]).astype(np.int64)


def mu_weights(counts: np.ndarray) -> np.ndarray:
    """w_j = round(2^30 / count_j) in integers: floor((2^31 + c) / (2 c))."""
    c = np.asarray(counts, dtype=np.int64)
    assert int(c.min()) >= 1
    return ((1 << (W_BITS + 1)) + c) // (2 * c)


def decode(m: Sequence[int], log_n: int, scale: float) -> np.ndarray:
    """Real parts of the slots: sum_i m_i cos(pi i g_j / N) / scale (floating point; tests only)."""
    n = 1 << log_n
    g = galois_5(n)
    mm = np.array([float(v) for v in m])
    out = np.empty(n // 2)
    for j0 in range(0, n // 2, 256):
        gj = g[j0:j0 + 256]
        ang = (np.arange(n, dtype=np.int64)[None, :] * gj[:, None]) % (2 * n)
        out[j0:j0 + len(gj)] = np.cos(np.pi * ang / n) @ mm
    return out / scale


# ---------------------------------------------------------------- keys

@dataclasses.dataclass
class FoldKeys:
    P: FoldParams
    s: np.ndarray                                   # N ternary, weight 32
    amounts: Tuple[int, ...]                        # rotation amounts with keys
    relin: Dict[int, Dict[int, List[Tuple[np.ndarray, np.ndarray]]]]   # level -> z -> [(k_i, beta_i)]
    rot: Dict[int, Dict[int, List[Tuple[np.ndarray, np.ndarray]]]]     # amount -> z -> [(k_0, beta_0)]


def sparse_secret(seed: int, n: int) -> np.ndarray:
    t = np.arange(n, dtype=np.uint64)
    w = np.choose((t & np.uint64(3)).astype(np.int64),
                  prng.philox4x64_10(seed, prng.tag(FSEC, 0), t >> np.uint64(2), np.zeros_like(t), 0, 0))
    u = np.choose((t & np.uint64(3)).astype(np.int64),
                  prng.philox4x64_10(seed, prng.tag(FSEC, 1), t >> np.uint64(2), np.zeros_like(t), 0, 0))
    order = np.argsort(w, kind="stable")           # ascending words, ties by index
    s = np.zeros(n, dtype=np.int64)
    for pos in order[:H_WEIGHT]:
        s[pos] = -1 if int(u[pos]) & 1 else 1
    return s


def automorphism(a: np.ndarray, g: int, q: int | None = None) -> np.ndarray:
    """a(X^g) in Z[X]/(X^N + 1) (g odd): X^i -> (-1)^floor(i g / N) X^(i g mod N)."""
    n = len(a)
    out = np.zeros(n, dtype=object if q is None else np.int64)
    for i in range(n):
        t = i * g % (2 * n)
        v = int(a[i])
        if t >= n:
            out[t - n] = -v if q is None else (-v) % q
        else:
            out[t] = v if q is None else v % q
    return out


def rot_galois(P: FoldParams, r: int) -> int:
    """Rot_r (slot i -> slot i + r) is X -> X^(5^-r): 5^(N/2 - r) mod 2N."""
    return pow(5, (P.slots - r) % P.slots, 2 * P.n)


def rot_amounts(k: int, rho: int) -> Tuple[int, ...]:
    """Rotations a fold of blocks of rho ciphertexts uses: 1 .. k-1 and r k for 1 <= r < ceil(rho / k)."""
    groups = -(-rho // k)
    return tuple(range(1, min(k, rho))) + tuple(r * k for r in range(1, groups))


def _square(s: np.ndarray) -> np.ndarray:
    n = len(s)
    full = np.convolve(s, s)
    out = full[:n].copy()
    out[: n - 1] -= full[n:]
    return out


def _ks_key(P: FoldParams, seed: int, kappa: int, level: int, s: np.ndarray, s_from: np.ndarray):
    """Key switching key from s_from to s at `level`: z -> [(k_i, beta_i)] over q_0 .. q_level, p."""
    n = P.n
    t = np.arange(n, dtype=np.uint64)
    primes = P.moduli(level)
    Ql = P.Q(level)
    out = {}
    for z in primes + [P.p]:
        row = []
        for i, qi in enumerate(primes):
            col = np.full(n, kappa * 8 + i, dtype=np.uint64)
            ka = prng.uniform_mod(seed, FKA, P.sid(z), t, col, z)
            e = prng.gaussian(seed, FKE, 0, t, col)
            g = P.p * (Ql // qi) % z
            beta = (-negmul_mod(s % z, ka, z) + g * s_from + e) % z          # |g s_from| < 2^41
            row.append((ka, beta))
        out[z] = row
    return out


def fold_keygen(P: FoldParams, seed: int, amounts: Sequence[int]) -> FoldKeys:
    s = sparse_secret(seed, P.n)
    s2 = _square(s)                                # |s^2| <= 32 coefficientwise
    relin = {lvl: _ks_key(P, seed, lvl - 1, lvl, s, s2) for lvl in (1, 2, 3)}
    rot = {}
    for a_idx, r in enumerate(amounts):
        rot[r] = _ks_key(P, seed, 3 + a_idx, ROT_LEVEL, s, automorphism(s, rot_galois(P, r)).astype(np.int64))
    return FoldKeys(P, s, tuple(amounts), relin, rot)


# ---------------------------------------------------------------- ciphertext arithmetic
# A ciphertext: (level, b, a) with b, a dicts modulus -> int64 coefficient residues.

Ct = Tuple[int, Dict[int, np.ndarray], Dict[int, np.ndarray]]


def encrypt(FK: FoldKeys, ip: np.ndarray, seed: int, index: int) -> Ct:
    """Input ciphertext `index`: the inner products ip (N/2 integers) at scale 2^20, level 4."""
    P = FK.P
    n = P.n
    t = np.arange(n, dtype=np.uint64)
    col = np.full(n, index, dtype=np.uint64)
    m = encode(ip, P.log_n, LOG_IN)
    e = prng.gaussian(seed, FXE, 0, t, col)
    b, a = {}, {}
    for z in P.moduli(LEVELS):
        a[z] = prng.uniform_mod(seed, FXA, P.sid(z), t, col, z)
        b[z] = (-negmul_mod(FK.s % z, a[z], z) + m + e) % z
    return (LEVELS, b, a)


def decrypt(FK: FoldKeys, ct: Ct) -> List[int]:
    """Centered b + a s mod Q_level (Python integers, by CRT over the level's primes)."""
    lvl, b, a = ct
    primes = FK.P.moduli(lvl)
    res = {z: (b[z] + negmul_mod(FK.s % z, a[z], z)) % z for z in primes}
    Q = FK.P.Q(lvl)
    out = []
    for i in range(FK.P.n):
        x = 0
        for z in primes:
            Mi = Q // z
            x += int(res[z][i]) * Mi * pow(Mi, -1, z)
        out.append(centered(x, Q))
    return out


def mulc(x: np.ndarray, c: int, z: int) -> np.ndarray:
    """x c mod z in Python integers (the products exceed 64 bits)."""
    return (np.asarray(x, dtype=np.int64).astype(object) * (c % z) % z).astype(np.int64)


def rescale_by(res: Dict[int, np.ndarray], div: int, keep: List[int]) -> Dict[int, np.ndarray]:
    """RS_div: floor(x / div + 1/2) on residues: (x_z - [x_div]_centered) div^-1 mod z for z in keep."""
    xc = np.array([centered(int(v), div) for v in res[div]], dtype=np.int64)
    return {z: mulc((res[z] - xc) % z, pow(div % z, -1, z), z) for z in keep}


def rescale(P: FoldParams, ct: Ct) -> Ct:
    lvl, b, a = ct
    keep = P.moduli(lvl - 1)
    ql = P.q[lvl]
    return (lvl - 1, rescale_by(b, ql, keep), rescale_by(a, ql, keep))


def drop(P: FoldParams, ct: Ct, level: int) -> Ct:
    """The same ciphertext modulo fewer primes (scale unchanged)."""
    _, b, a = ct
    keep = P.moduli(level)
    return (level, {z: b[z] for z in keep}, {z: a[z] for z in keep})


def add(ct1: Ct, ct2: Ct) -> Ct:
    assert ct1[0] == ct2[0]
    l, b1, a1 = ct1
    _, b2, a2 = ct2
    return (l, {z: (b1[z] + b2[z]) % z for z in b1}, {z: (a1[z] + a2[z]) % z for z in a1})


def mul_const(ct: Ct, c: int) -> Ct:
    l, b, a = ct
    return (l, {z: mulc(b[z], c, z) for z in b}, {z: mulc(a[z], c, z) for z in a})


def add_const(ct: Ct, c: int) -> Ct:
    l, b, a = ct
    nb = {}
    for z in b:
        v = b[z].copy()
        v[0] = (v[0] + c) % z
        nb[z] = v
    return (l, nb, dict(a))


def mul_plain(ct: Ct, m: np.ndarray) -> Ct:
    l, b, a = ct
    return (l, {z: negmul_mod(m % z, b[z], z) for z in b}, {z: negmul_mod(m % z, a[z], z) for z in a})


def key_switch_sums(P: FoldParams, level: int, x: Dict[int, np.ndarray], key) -> Tuple[Dict, Dict]:
    """sum_i d_i K_i modulo Q_l p, d_i = [x (Q_l/q_i)^-1]_{q_i}: (B, A) before the division by p."""
    primes = P.moduli(level)
    Ql = P.Q(level)
    dig = [mulc(x[qi], pow((Ql // qi) % qi, -1, qi), qi) for qi in primes]
    A, B = {}, {}
    for z in primes + [P.p]:
        acc_a = np.zeros(P.n, dtype=np.int64)
        acc_b = np.zeros(P.n, dtype=np.int64)
        for i in range(len(primes)):
            ka, beta = key[z][i]
            acc_a = (acc_a + negmul_mod(dig[i] % z, ka, z)) % z
            acc_b = (acc_b + negmul_mod(dig[i] % z, beta, z)) % z
        A[z], B[z] = acc_a, acc_b
    return B, A


def key_switch(P: FoldParams, level: int, x: Dict[int, np.ndarray], key) -> Tuple[Dict, Dict]:
    """(B, A) with B + A s = x s_from + small: RS_p(sum_i d_i K_i), d_i = [x (Q_l/q_i)^-1]_{q_i}."""
    primes = P.moduli(level)
    B, A = key_switch_sums(P, level, x, key)
    return rescale_by(B, P.p, primes), rescale_by(A, P.p, primes)


def rescale_by_two(res: Dict[int, np.ndarray], p: int, ql: int, keep: List[int]) -> Dict[int, np.ndarray]:
    """RS_{p q_l}: floor(x / (p q_l) + 1/2) on residues over keep + [q_l, p]: the centered value c of x modulo
    D = p q_l by the CRT of its residues modulo p and q_l, then (x_z - c) D^-1 mod z for z in keep."""
    D = p * ql
    pinv = pow(p, -1, ql)
    c = []
    for a, b in zip(res[p], res[ql]):
        v = int(a) + p * ((int(b) - int(a)) * pinv % ql)      # = a mod p, = b mod q_l, in [0, D)
        c.append(centered(v, D))
    c = np.array(c, dtype=object)
    out = {}
    for z in keep:
        inv = pow(D % z, -1, z)
        out[z] = np.array([(int(x) - int(cv)) * inv % z for x, cv in zip(res[z], c)], dtype=np.int64)
    return out


def mul(FK: FoldKeys, ct1: Ct, ct2: Ct, rescaled: bool = True) -> Ct:
    """Product with relinearisation.  Rescaled (the default): the key switch's sums and the tensor's d0, d1
    times p are divided by p q_l in one rounding, RS_{p q_l}(p (d0, d1) + sum_i d_i K_i), which lands at level
    l - 1 as RS_{q_l} of the relinearised product does; otherwise the relinearised product at level l,
    (d0, d1) + RS_p(sum_i d_i K_i)."""
    P = FK.P
    l, b1, a1 = ct1
    l2, b2, a2 = ct2
    assert l == l2 and l >= 1
    d0, d1, d2 = {}, {}, {}
    for z in P.moduli(l):
        d0[z] = negmul_mod(b1[z], b2[z], z)
        d1[z] = (negmul_mod(a1[z], b2[z], z) + negmul_mod(a2[z], b1[z], z)) % z
        d2[z] = negmul_mod(a1[z], a2[z], z)
    if not rescaled:
        B, A = key_switch(P, l, d2, FK.relin[l])
        return (l, {z: (d0[z] + B[z]) % z for z in d0}, {z: (d1[z] + A[z]) % z for z in d1})
    B, A = key_switch_sums(P, l, d2, FK.relin[l])
    primes = P.moduli(l)
    XB = {z: (B[z] + mulc(d0[z], P.p, z)) % z for z in primes}
    XA = {z: (A[z] + mulc(d1[z], P.p, z)) % z for z in primes}
    XB[P.p], XA[P.p] = B[P.p], A[P.p]
    keep = primes[:-1]
    return (l - 1, rescale_by_two(XB, P.p, P.q[l], keep), rescale_by_two(XA, P.p, P.q[l], keep))


def rotate(FK: FoldKeys, ct: Ct, r: int) -> Ct:
    """Rot_r at level 1: (sigma(b) + B, A) with (B, A) = KS(sigma(a)) to s."""
    P = FK.P
    l, b, a = ct
    assert l == ROT_LEVEL
    g = rot_galois(P, r)
    primes = P.moduli(l)
    sb = {z: automorphism(b[z], g, z) for z in primes}
    sa = {z: automorphism(a[z], g, z) for z in primes}
    B, A = key_switch(P, l, sa, FK.rot[r])
    return (l, {z: (sb[z] + B[z]) % z for z in primes}, A)


# ---------------------------------------------------------------- scales and the polynomial

def rnd(v: float) -> int:
    return math.floor(v + 0.5)


@dataclasses.dataclass(frozen=True)
class Schedule:
    S1: float
    S2: float
    S4: float
    F: float
    U: float
    T3: float
    T1: float
    G: float                  # scale of f at level 1: F q_1
    k: Tuple[int, ...]        # integer constants k_0 .. k_7


def schedule(P: FoldParams) -> Schedule:
    """The scales of the powers and the integer constants of f.  Each scale is one product and one
    quotient of doubles, in this order, so that another implementation reaches the same constants."""
    q1, q2, q3, q4 = (float(P.q[i]) for i in (1, 2, 3, 4))
    S1 = float(1 << (LOG_IN + LOG_MU)) / q4               # x = RS_{q_4}(ct * mu), level 3
    S2 = (S1 * S1) / q3                                    # x^2, level 2
    S4 = (S2 * S2) / q2                                    # x^4, level 1
    F = float(1 << LOG_F)                                  # the folded result, level 0
    G = F * q1                                             # f at level 1 (exact: 24 + 23 bits)
    U = G / S4                                             # x^4 * inner at level 1 has scale G
    T3 = (U * q2) / S2                                     # x^2 * L3 at level 1 has scale U
    T1 = (G * q2) / S2                                     # x^2 * L1 at level 1 has scale G
    E7 = (T3 * q3) / S1                                    # c7 x at level 2 has scale T3
    E3 = (T1 * q3) / S1
    E5 = (U * q3) / S1
    E1 = (G * q3) / S1
    c = COEFFS
    k = (rnd(c[0] * G), rnd(c[1] * E1), rnd(c[2] * T1), rnd(c[3] * E3),
         rnd(c[4] * U), rnd(c[5] * E5), rnd(c[6] * T3), rnd(c[7] * E7))
    return Schedule(S1, S2, S4, F, U, T3, T1, G, k)


def normalise(FK: FoldKeys, ct: Ct, counts: np.ndarray) -> Ct:
    """x = RS_{q_4}(ct (.) Ecd(1 / counts)) at level 3."""
    m = encode(mu_weights(counts), FK.P.log_n, LOG_MU - W_BITS)
    return rescale(FK.P, mul_plain(ct, m))


def poly_f(FK: FoldKeys, x: Ct) -> Ct:
    """f(x) at level 1, scale G = F q_1, for x at level 3, scale S1."""
    P = FK.P
    k = schedule(P).k
    x2 = mul(FK, x, x)                                                    # level 2
    L3 = add_const(rescale(P, mul_const(x, k[7])), k[6])                  # level 2
    L1 = add_const(rescale(P, mul_const(x, k[3])), k[2])                  # level 2
    L2 = add_const(drop(P, rescale(P, mul_const(x, k[5])), 1), k[4])      # level 1
    L0 = add_const(drop(P, rescale(P, mul_const(x, k[1])), 1), k[0])      # level 1
    x4 = mul(FK, x2, x2)                                                  # level 1
    inner = add(mul(FK, x2, L3), L2)                                      # level 1
    t1 = mul(FK, x2, L1)                                                  # level 1
    t4 = mul(FK, x4, inner, rescaled=False)                               # level 1, scale G
    return add(add(L0, t1), t4)


def fold(FK: FoldKeys, cts: List[Ct], counts: np.ndarray, rho: int) -> List[Ct]:
    """Blocks of rho ciphertexts (len(cts) a multiple of rho) -> ceil(rho / k) folded ciphertexts per
    block, block-major."""
    P = FK.P
    n = len(cts)
    assert n % rho == 0 and rho <= P.slots
    out = []
    for blk in range(n // rho):
        for r in range(-(-rho // P.k)):
            acc = None
            for rp in range(min(P.k, rho - r * P.k)):
                c = blk * rho + r * P.k + rp
                y = poly_f(FK, normalise(FK, cts[c], counts[c]))
                if rp:
                    y = rotate(FK, y, rp)
                acc = y if acc is None else add(acc, y)
            if r:
                acc = rotate(FK, acc, r * P.k)
            out.append(rescale(P, acc))
    return out


def f_plain(x: np.ndarray) -> np.ndarray:
    """The folding polynomial on plain values."""
    return np.polyval(np.array(COEFFS[::-1]), x)


def fold_plain(ip: np.ndarray, counts: np.ndarray, rho: int, k: int) -> np.ndarray:
    """What the folded ciphertexts decrypt to: sum_r' roll(f(ip / counts), r k + r') per group."""
    n, slots = ip.shape
    out = []
    for blk in range(n // rho):
        for r in range(-(-rho // k)):
            acc = np.zeros(slots)
            for rp in range(min(k, rho - r * k)):
                c = blk * rho + r * k + rp
                acc += np.roll(f_plain(ip[c] / counts[c]), r * k + rp)
            out.append(acc)
    return np.array(out)
