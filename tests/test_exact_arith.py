"""Exact integer results that the kernels reach through floating point or multiply-high quotients.

The helpers of paper_2601_17561_amd/csrc/hfe_exact.h are host and device functions; the CPU build
tests/native/libhfe_exact_check.so applies each of them, as the kernels call it, to operands chosen
here: random ones, the extremes of each stated range, and operands next to the places where a
quotient estimate can be off (products next to multiples of the modulus, sums at the CRT's 1/4
margin).  Every result is compared with Python integer arithmetic; the exhaustive sweeps compare with
C's integer remainder inside the harness.

  mulmod_d      a w mod q in fp64 (the NTT butterflies), q < 2^36
  mulmod_c_d, reduce_c_d, ct_butterfly_c
                the signed product (|a| <= 16q, centered result), reduction and butterfly of the
                FormatSwitch transforms, and a whole transform built from them
  mod_small     x mod m by multiply-high, x < 2^24, 2 <= m <= 256 (every x, every m)
  mod_u32       x mod m by multiply-high with one correction, x < 2^32, m <= 2^16 (the chain's n^2)
  mod_f64       x mod m by an fp64 quotient, |x| < 2^48, m < 2^24
  balanced_mod  the RNS form's int8 residues, |x| < 2^40
  p2_digits     the n^2 form's digits M + n M', |x| < 2^48
  rns_acc_mod   the RNS contraction epilogue, every int32 sum (strided sweep and extremes)
  p2_acc_mod    the n^2 contraction epilogue, int32 sums G0, G1
  CRT           the fp32 fractional-sum CRT of both forms, |S| <= M/4, up to 16 moduli / 8 bases
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import params as OP

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "libhfe_exact_check.so")
if not os.path.exists(LIB):  # pragma: no cover
    pytest.fail(f"{LIB} is missing: build it with `python paper_2601_17561_amd/build.py`", pytrace=False)
_L = ctypes.CDLL(LIB)
_p = ctypes.c_void_p
_L.xc_mod_small_sweep.restype = ctypes.c_int64
_L.xc_mod_small_sweep.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
_L.xc_rns_acc_mod_sweep.restype = ctypes.c_int64
_L.xc_rns_acc_mod_sweep.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
for _name, _args in {
        "xc_mulmod_d": [_p, _p, ctypes.c_int64, ctypes.c_uint64, _p],
        "xc_mulmod_c_d": [_p, _p, ctypes.c_int64, ctypes.c_uint64, _p],
        "xc_reduce_c_d": [_p, ctypes.c_int64, ctypes.c_uint64, _p],
        "xc_ntt_signed": [_p, _p, ctypes.c_int, ctypes.c_uint64, _p],
        "xc_slot_encode": [_p, ctypes.c_int, ctypes.c_int, _p],
        "xc_mod_small": [_p, ctypes.c_int64, ctypes.c_uint32, _p],
        "xc_mod_f64": [_p, ctypes.c_int64, ctypes.c_int64, _p],
        "xc_balanced_mod": [_p, ctypes.c_int64, ctypes.c_int, _p],
        "xc_p2_digits": [_p, ctypes.c_int64, ctypes.c_int, _p, _p],
        "xc_rns_acc_mod": [_p, ctypes.c_int64, ctypes.c_int, _p],
        "xc_p2_acc_mod": [_p, _p, ctypes.c_int64, ctypes.c_int, _p],
        "xc_p2_digits_n": [_p, ctypes.c_int64, ctypes.c_int32, _p, _p],
        "xc_p2_acc_mod_n": [_p, _p, ctypes.c_int64, ctypes.c_int32, _p],
        "xc_crt": [_p, ctypes.c_int64, ctypes.c_int, _p, _p, _p, _p, ctypes.c_uint64, ctypes.c_uint64,
                   ctypes.c_uint64, ctypes.c_int, _p, _p]}.items():
    getattr(_L, _name).argtypes = _args
    getattr(_L, _name).restype = None
_L.xc_ntt_signed.restype = ctypes.c_int64
_L.xc_intt_signed.restype = ctypes.c_int64
_L.xc_intt_signed.argtypes = [_p, _p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _p]
_L.xc_mod_u32_sweep.restype = ctypes.c_int64
_L.xc_mod_u32_sweep.argtypes = [ctypes.c_uint32, ctypes.c_int64]

# The moduli tables of the library (hfe_exact.h); their values are fixed by the paper's ranges
# (RNS: pairwise coprime, <= 256; n^2: primes 127 <= n <= 253) and checked below.
RNS_MODS = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191]
P2_BASES = [251, 241, 239, 233, 229, 227, 223, 211]


def _ptr(a):
    return a.ctypes.data


def _largest_prime_below(x):
    q = x - 1
    while not OP.is_prime(q):
        q -= 1
    return q


def test_tables_match_the_header():
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_2601_17561_amd", "csrc", "hfe_exact.h")).read()
    assert "{" + ", ".join(str(m) for m in RNS_MODS[:8]) + "," in src.replace("\n", " ").replace("  ", "")
    assert "{" + ", ".join(str(n) for n in P2_BASES) + "}" in src
    from math import gcd
    assert all(gcd(a, b) == 1 for i, a in enumerate(RNS_MODS) for b in RNS_MODS[i + 1:])
    assert all(OP.is_prime(n) and 127 <= n <= 253 for n in P2_BASES)


@pytest.mark.parametrize("q", OP.ntt_primes(9) + [_largest_prime_below(1 << 36), (1 << 20) + 7])
def test_mulmod_d_exact(q):
    rng = np.random.default_rng(q % 1000)
    n = 200_000
    a = rng.integers(0, q, n, dtype=np.uint64)
    w = rng.integers(0, q, n, dtype=np.uint64)
    ext = [0, 1, 2, q - 1, q - 2, (q - 1) // 2, (q + 1) // 2]
    ea, ew = np.meshgrid(ext, ext)
    # products next to multiples of q: a = t w^-1 mod q gives a w = t (mod q) for t near 0 and q
    ww = rng.integers(1, q, 20_000).tolist()
    tt = [0, 1, 2, 3, q - 1, q - 2, q - 3]
    near_a = [(t * pow(x, -1, q)) % q for x in ww for t in tt]
    near_w = [x for x in ww for _ in tt]
    A = np.concatenate([a, ea.ravel().astype(np.uint64), np.array(near_a, dtype=np.uint64)])
    Wv = np.concatenate([w, ew.ravel().astype(np.uint64), np.array(near_w, dtype=np.uint64)])
    out = np.empty_like(A)
    _L.xc_mulmod_d(_ptr(A), _ptr(Wv), len(A), q, _ptr(out))
    want = [int(x) * int(y) % q for x, y in zip(A.tolist(), Wv.tolist())]
    assert out.tolist() == want


@pytest.mark.parametrize("q", OP.ntt_primes(4) + [_largest_prime_below(1 << 36)])
def test_signed_product_and_reduction(q):
    """The signed arithmetic of the FormatSwitch transforms: a w congruent mod q and at most
    (1/2 + 2^-11) q in magnitude for |a| <= 16q; x - q rint(x / q) then the residue in [0, q)."""
    rng = np.random.default_rng(q % 991)
    n = 200_000
    lim = 16 * q
    ext = [0, 1, -1, q - 1, -(q - 1), q, -q, 2 * q + 1, lim, -lim, lim - 1, -(lim - 1), q // 2, -(q // 2)]
    wx = [0, 1, 2, q - 1, q - 2, (q - 1) // 2, (q + 1) // 2]
    a = np.concatenate([rng.integers(-lim, lim + 1, n, dtype=np.int64), np.repeat(ext, len(wx)).astype(np.int64)])
    w = np.concatenate([rng.integers(0, q, n, dtype=np.uint64), np.tile(wx, len(ext)).astype(np.uint64)])
    # products next to half-multiples of q (where the rounded quotient may go either way)
    ww = rng.integers(1, q, 20_000).tolist()
    near = [(((t * pow(x, -1, q)) % q) + k * q, x) for x in ww for t in (q // 2, q // 2 + 1, 0, 1) for k in (-16, 3, 15)]
    a = np.concatenate([a, np.array([u for u, _ in near], dtype=np.int64)])
    w = np.concatenate([w, np.array([v for _, v in near], dtype=np.uint64)])
    out = np.empty_like(a)
    _L.xc_mulmod_c_d(_ptr(a), _ptr(w), len(a), q, _ptr(out))
    bound = q // 2 + q // 2048 + 1
    assert all(abs(o) <= bound and (o - x * y) % q == 0 for x, y, o in zip(a.tolist(), w.tolist(), out.tolist()))
    x = np.concatenate([rng.integers(-(1 << 47) + 1, 1 << 47, n, dtype=np.int64), np.array(ext, dtype=np.int64)])
    r = np.empty(len(x), dtype=np.uint64)
    _L.xc_reduce_c_d(_ptr(x), len(x), q, _ptr(r))
    assert r.tolist() == [v % q for v in x.tolist()]


@pytest.mark.parametrize("logn", [7, 13, 14])
def test_signed_transform_equals_the_negacyclic_evaluation(logn):
    """A whole forward transform through the signed butterflies (inputs in [0, 2q), the digits' range)
    equals the exact one (the integer transform reduced mod q), and its values stay below 9.1q."""
    q = OP.ntt_primes(1)[0]
    n = 1 << logn
    g = 2
    while pow(g, (q - 1) // 2, q) == 1:     # a quadratic non-residue: psi = g^((q-1)/2n) has order 2n
        g += 1
    psi = pow(g, (q - 1) // (2 * n), q)
    assert pow(psi, n, q) == q - 1
    brv = [int(format(i, f"0{logn}b")[::-1], 2) for i in range(n)]
    w = np.array([pow(psi, brv[i], q) for i in range(n)], dtype=np.uint64)
    rng = np.random.default_rng(logn)
    x = rng.integers(0, 2 * q, n, dtype=np.int64)
    x[:4] = 2 * q - 1
    out = np.empty(n, dtype=np.uint64)
    big = _L.xc_ntt_signed(_ptr(x), _ptr(w), logn, q, _ptr(out))
    assert big < 9.1 * q
    xs = [int(v) for v in x.tolist()]
    # merged negacyclic transform: output i is the evaluation at psi^(2 brv(i) + 1)
    for i in list(range(0, n, max(1, n // 64))) + [n - 1]:
        z = pow(psi, 2 * brv[i] + 1, q)
        assert int(out[i]) == sum(c * pow(z, t, q) for t, c in enumerate(xs)) % q


@pytest.mark.parametrize("m", [255, 256, 16129, 38809, 39601, 44521, 49729, 51529, 57121, 63001, 65536])
def test_mod_u32_exact(m):
    """x mod m for 32-bit x and the n^2 moduli (127^2 .. 251^2 and the default chain's): every x < 2^24,
    every x within 3 of a multiple of m, 2^32 - 1, and 2 M pseudo-random x."""
    assert _L.xc_mod_u32_sweep(m, 2_000_000) == 0


@pytest.mark.parametrize("logn", [7, 12, 13, 14])
def test_signed_inverse_transform_inverts_the_forward_one(logn):
    """The signed inverse transform of the kernels (rounds from centered representatives) applied to the
    exact forward transform returns the input, for inputs of any sign and size up to 2^40, and keeps every
    value inside a round below 8.02q."""
    q = OP.ntt_primes(1)[0]
    n = 1 << logn
    g = 2
    while pow(g, (q - 1) // 2, q) == 1:
        g += 1
    psi = pow(g, (q - 1) // (2 * n), q)
    brv = [int(format(i, f"0{logn}b")[::-1], 2) for i in range(n)]
    ipsi = pow(psi, q - 2, q)
    iw = np.array([pow(ipsi, brv[i], q) for i in range(n)], dtype=np.uint64)
    w = np.array([pow(psi, brv[i], q) for i in range(n)], dtype=np.uint64)
    rng = np.random.default_rng(logn + 100)
    x = rng.integers(0, q, n, dtype=np.int64)
    xs = [int(v) for v in x.tolist()]
    # the forward transform (pinned against the evaluation at psi^(2 brv(i) + 1) above), then the inputs
    # of the inverse spread over representatives of both signs and large magnitude
    fwd = np.empty(n, dtype=np.uint64)
    _L.xc_ntt_signed(_ptr(x), _ptr(w), logn, q, _ptr(fwd))
    ev = [int(v) for v in fwd.tolist()]
    k = rng.integers(-(1 << 4), 1 << 4, n)
    inp = np.array([v + int(t) * q for v, t in zip(ev, k.tolist())], dtype=np.int64)
    out = np.empty(n, dtype=np.uint64)
    big = _L.xc_intt_signed(_ptr(inp), _ptr(iw), logn, q, pow(n, q - 2, q), _ptr(out))
    assert big < 8.02 * q
    assert out.tolist() == xs


def test_mod_small_exact_for_every_operand():
    for m in range(2, 257):
        assert _L.xc_mod_small_sweep(m, 1 << 24) == 0, m
    for n in P2_BASES:                                  # the n^2 digits use it below 2^17
        assert _L.xc_mod_small_sweep(n, 1 << 17) == 0, n
    x = np.array([0, 1, (1 << 24) - 1, (1 << 24) - 2, 255, 256, 65535], dtype=np.uint32)
    for m in RNS_MODS:
        out = np.empty_like(x)
        _L.xc_mod_small(_ptr(x), len(x), m, _ptr(out))
        assert out.tolist() == [int(v) % m for v in x]


@pytest.mark.parametrize("m", P2_BASES + [n * n for n in P2_BASES] + [2, 3, (1 << 24) - 1, (1 << 24) - 3])
def test_mod_f64_exact(m):
    rng = np.random.default_rng(m)
    lim = (1 << 48) - 1
    x = rng.integers(-lim, lim, 100_000, dtype=np.int64)
    k = rng.integers(-(lim // m), lim // m, 20_000, dtype=np.int64)
    near = np.concatenate([k * m - 1, k * m, k * m + 1])
    near = near[np.abs(near) <= lim]
    X = np.concatenate([x, near, np.array([0, 1, -1, lim, -lim, m, -m, m - 1, 1 - m], dtype=np.int64)])
    out = np.empty_like(X)
    _L.xc_mod_f64(_ptr(X), len(X), m, _ptr(out))
    assert out.tolist() == [int(v) % m for v in X.tolist()]


@pytest.mark.parametrize("j", range(16))
def test_balanced_mod_exact(j):
    m = RNS_MODS[j]
    rng = np.random.default_rng(100 + j)
    lim = (1 << 40) - 1
    k = rng.integers(-(lim // m), lim // m, 20_000, dtype=np.int64)
    X = np.concatenate([rng.integers(-lim, lim, 100_000, dtype=np.int64), k * m - 1, k * m, k * m + 1,
                        np.array([0, 1, -1, lim, -lim, m // 2, -(m // 2), (m + 1) // 2, -((m + 1) // 2)],
                                 dtype=np.int64)])
    X = X[np.abs(X) <= lim]
    out = np.empty(len(X), dtype=np.int32)
    _L.xc_balanced_mod(_ptr(X), len(X), j, _ptr(out))
    lo, hi = -(m // 2), (m + 1) // 2 - 1
    assert out.min() >= lo and out.max() <= hi
    assert all((int(r) - int(v)) % m == 0 for r, v in zip(out.tolist(), X.tolist()))


@pytest.mark.parametrize("j", range(8))
def test_p2_digits_exact(j):
    n = P2_BASES[j]
    n2 = n * n
    h = (n - 1) // 2
    rng = np.random.default_rng(200 + j)
    lim = (1 << 48) - 1
    r = np.arange(n2, dtype=np.int64)                  # every residue mod n^2 ...
    k = rng.integers(-(lim // n2) + 1, lim // n2 - 1, n2, dtype=np.int64)
    X = np.concatenate([r, r + k * n2, -r, rng.integers(-lim, lim, 50_000, dtype=np.int64),
                        np.array([lim, -lim, 0, 1, -1], dtype=np.int64)])   # ... at random offsets
    M = np.empty(len(X), dtype=np.int32)
    Mp = np.empty(len(X), dtype=np.int32)
    _L.xc_p2_digits(_ptr(X), len(X), j, _ptr(M), _ptr(Mp))
    assert np.abs(M).max() <= h and np.abs(Mp).max() <= h
    assert all((int(a) + n * int(b) - int(x)) % n2 == 0 for a, b, x in zip(M.tolist(), Mp.tolist(), X.tolist()))


@pytest.mark.parametrize("j", range(16))
def test_rns_epilogue_exact_over_int32(j):
    m = RNS_MODS[j]
    assert _L.xc_rns_acc_mod_sweep(j, -(1 << 31), 997, ((1 << 32) - 1) // 997 + 1) == 0
    assert _L.xc_rns_acc_mod_sweep(j, (1 << 31) - 5000, 1, 5000) == 0
    assert _L.xc_rns_acc_mod_sweep(j, -(1 << 31), 1, 5000) == 0
    S = np.array([-(1 << 31), -(1 << 31) + 1, -1, 0, 1, (1 << 31) - 1, m, -m, m - 1, 1 - m], dtype=np.int32)
    out = np.empty(len(S), dtype=np.uint32)
    _L.xc_rns_acc_mod(_ptr(S), len(S), j, _ptr(out))
    assert out.tolist() == [int(s) % m for s in S.tolist()]


@pytest.mark.parametrize("j", range(8))
def test_p2_epilogue_exact(j):
    n = P2_BASES[j]
    rng = np.random.default_rng(300 + j)
    ext = np.array([-(1 << 31), -(1 << 31) + 1, -1, 0, 1, (1 << 31) - 1, n, -n, n * n, -n * n], dtype=np.int32)
    g0 = np.concatenate([rng.integers(-(1 << 31), 1 << 31, 200_000, dtype=np.int64).astype(np.int32),
                         np.repeat(ext, len(ext))])
    g1 = np.concatenate([rng.integers(-(1 << 31), 1 << 31, 200_000, dtype=np.int64).astype(np.int32),
                         np.tile(ext, len(ext))])
    out = np.empty(len(g0), dtype=np.uint32)
    _L.xc_p2_acc_mod(_ptr(g0), _ptr(g1), len(g0), j, _ptr(out))
    assert out.tolist() == [(int(a) + n * int(b)) % (n * n) for a, b in zip(g0.tolist(), g1.tolist())]


def _crt_case(moduli, q, S, p2):
    M = 1
    for m in moduli:
        M *= m
    nm = len(moduli)
    s = np.array([[int(x) % m for x in S] for m in moduli], dtype=np.uint32)
    inv = np.array([pow(M // m % m, -1, m) for m in moduli], dtype=np.uint32)
    rcp = np.array([np.float32(1.0) / np.float32(m) for m in moduli], dtype=np.float32)
    Mj = np.array([(M // m) % q for m in moduli], dtype=np.uint64)
    m_arr = np.array(moduli, dtype=np.uint32)
    out = np.empty(len(S), dtype=np.uint64)
    a_out = np.empty(len(S), dtype=np.uint64)
    _L.xc_crt(_ptr(s), len(S), nm, _ptr(m_arr), _ptr(inv), _ptr(rcp), _ptr(Mj), M % q, q, (1 << 64) // q,
              1 if p2 else 0, _ptr(out), _ptr(a_out))
    for e, x in enumerate(S):
        y = [int(s[j, e]) * int(inv[j]) % moduli[j] for j in range(nm)]
        a = (sum(yj * (M // m) for yj, m in zip(y, moduli)) - x) // M
        assert int(a_out[e]) == a, (nm, x)
        assert int(out[e]) == x % q, (nm, x)


@pytest.mark.parametrize("form", ["rns", "p2"])
def test_crt_fractional_sum_exact_at_the_quarter_margin(form):
    """Every prefix of the moduli (RNS: 1..16, n^2: the squares of 1..8 bases), with |S| <= M/4: the
    extremes +-M/4, +-(M/4 - 1), 0, +-1 and random S."""
    q = OP.ntt_primes(1)[0]
    mods = RNS_MODS if form == "rns" else [n * n for n in P2_BASES]
    rng = np.random.default_rng(7)
    for nm in range(1, len(mods) + 1):
        moduli = mods[:nm]
        M = 1
        for m in moduli:
            M *= m
        B = M // 4
        S = [B, -B, B - 1, -(B - 1), 0, 1, -1] + [int(rng.integers(0, 1 << 62)) * B // (1 << 62) *
                                                  (1 if rng.random() < 0.5 else -1) for _ in range(500)]
        _crt_case(moduli, q, S, form == "p2")


CHAIN_BASES = [n for n in range(253, 126, -1) if all(n % d for d in range(2, int(n ** 0.5) + 1))]


@pytest.mark.parametrize("n", CHAIN_BASES)
def test_chain_digits_and_epilogue_exact_for_every_base(n):
    """The n^2 modulus chain's split (centered residues mod n^2, |x| < n^2) and contraction epilogue with
    the constants its kernels take, for each of the 24 primes 127 <= n <= 253: every residue, and
    random and extreme int32 sums."""
    n2 = n * n
    h = (n - 1) // 2
    X = np.concatenate([np.arange(-(n2 // 2), n2 // 2 + 1, dtype=np.int64), np.array([n2, -n2], dtype=np.int64)])
    M = np.empty(len(X), dtype=np.int32)
    Mp = np.empty(len(X), dtype=np.int32)
    _L.xc_p2_digits_n(_ptr(X), len(X), n, _ptr(M), _ptr(Mp))
    assert np.abs(M).max() <= h and np.abs(Mp).max() <= h
    assert np.all((M.astype(np.int64) + n * Mp.astype(np.int64) - X) % n2 == 0)
    rng = np.random.default_rng(n)
    ext = np.array([-(1 << 31), -(1 << 31) + 1, -1, 0, 1, (1 << 31) - 1, n, -n, n2, -n2], dtype=np.int32)
    g0 = np.concatenate([rng.integers(-(1 << 31), 1 << 31, 50_000, dtype=np.int64).astype(np.int32),
                         np.repeat(ext, len(ext))])
    g1 = np.concatenate([rng.integers(-(1 << 31), 1 << 31, 50_000, dtype=np.int64).astype(np.int32),
                         np.tile(ext, len(ext))])
    out = np.empty(len(g0), dtype=np.uint32)
    _L.xc_p2_acc_mod_n(_ptr(g0), _ptr(g1), len(g0), n, _ptr(out))
    want = (g0.astype(np.int64) + n * g1.astype(np.int64)) % n2
    assert np.array_equal(out.astype(np.int64), want)


@pytest.mark.parametrize("log_n,e", [(7, 20), (10, 10), (14, 10), (14, 20)])
def test_slot_encoder_matches_the_oracle_bit_for_bit(log_n, e):
    """The fold's slot encoder as the kernel runs it (hfe_slots.h, host build) takes the same rounding
    decisions as the oracle's encoder (oracle/fold.py, numpy): the same sequence of IEEE operations on the
    same tables.  Inner products (|w| <= 2^14) at scale 2^20 and normalisation weights (up to 2^30, with
    the dynamic range of counts from 1 to 2^14) at scale 2^10."""
    from oracle import fold as OF
    rng = np.random.default_rng(log_n + e)
    m = (1 << log_n) // 2
    if e == 20:
        w = rng.integers(-(1 << 14), 1 << 14, m)
    else:
        c = rng.integers(1, 1 << 14, m)
        w = ((1 << 31) + c) // (2 * c)
    w = w.astype(np.int64)
    out = np.empty(1 << log_n, dtype=np.int64)
    _L.xc_slot_encode(_ptr(w), log_n, e, _ptr(out))
    assert np.array_equal(out, OF.encode(w, log_n, e))
