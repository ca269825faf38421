"""The C-ABI library on the host (no GPU needed): symbols, host-side tables, validation.

* Every entry point declared in include/hfe.h is exported by libhfe.so.
* The library's quad-precision Gaussian table equals the oracle's exact decimal table.
* Default parameters pick the same primes the oracle derives independently.
* Invalid parameters and arguments are rejected with the documented status codes before
  any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

H = pytest.importorskip("paper_2601_17561_amd")
from oracle import params as OP  # noqa: E402
from oracle import prng  # noqa: E402


def _declared():
    src = open(os.path.join(ROOT, "include", "hfe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hfe_[a-z_0-9]+)\s*\(", src)) - {"hfe_alloc_fn", "hfe_dealloc_fn"})


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(H.LIB_PATH)
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(H.EXPORTED)


def test_cdt_table_matches_oracle():
    assert H.hfe_cdt_table() == prng.cdt_table()


@pytest.mark.parametrize("nq", [1, 3, 5, 8])
def test_default_params_primes_match_oracle(nq):
    P = H.hfe_default_params(14, 13, nq, 12800, 14336)
    q, p = P.primes()
    ref = OP.ntt_primes(nq + 1)
    assert p == ref[0] and q == ref[1:]
    assert P.gap_bits == 20 and (P.t_num, P.t_den) == (3, 8)


def _params(**kw):
    P = H.hfe_default_params(12, 12, 2, 1024, 256)
    for k, v in kw.items():
        setattr(P, k, v)
    return P


@pytest.mark.parametrize("kw,status", [
    (dict(log_n_db=0), -1),
    (dict(log_n_q=17), -1),                 # ring degrees 2^1 .. 2^16
    (dict(n_q_primes=0), -1),
    (dict(t_num=4, t_den=8), -1),
    (dict(t_den=0), -1),
    (dict(p=68718428161 - 2), -1),          # not prime
    (dict(p=12289), -1),                     # below 2^20
    (dict(gap_bits=1), -1),
    (dict(d2=1 << 19), -7),                  # d2 * Delta could reach Q/2
    (dict(d2=0), -1),
])
def test_invalid_params_rejected(kw, status):
    P = _params(**kw)
    with pytest.raises(H.HfeError) as e:
        H.hfe_keygen(P, 1)
    assert e.value.status == status


def test_prime_must_be_one_mod_2n():
    P = _params()
    # 2^36-ish prime that is 1 mod 2^12 but not 1 mod 2^13 is rejected for N = 2^12 rings
    q = None
    c = (1 << 35) + 1
    while q is None:
        if OP.is_prime(c) and (c - 1) % (1 << 12) == 0 and (c - 1) % (1 << 13) != 0:
            q = c
        c += 1 << 12
    P.q[1] = q
    with pytest.raises(H.HfeError) as e:
        H.hfe_keygen(P, 1)
    assert e.value.status == -1 and "1 mod 2N" in str(e.value)


def test_duplicate_primes_rejected():
    P = _params()
    P.q[1] = P.q[0]
    with pytest.raises(H.HfeError) as e:
        H.hfe_keygen(P, 1)
    assert e.value.status == -1


def test_null_arguments_rejected():
    lib = ctypes.CDLL(H.LIB_PATH)
    lib.hfe_export.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p,
                               ctypes.c_size_t, ctypes.c_void_p]
    assert lib.hfe_export(None, 0, 0, None, 0, None) == -1
    lib.hfe_encode.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.hfe_encode(None, None, 1, 8, None, 1, None, None) == -1
    lib.hfe_free.argtypes = [ctypes.c_void_p]
    lib.hfe_free(None)                       # NULL-safe
    lib.hfe_cdt_table.argtypes = [ctypes.c_void_p]
    assert lib.hfe_cdt_table(None) == -1


def test_one_hip_runtime_when_the_package_is_imported_before_torch():
    """Importing the package first must not load a second HIP runtime beside torch's."""
    import subprocess
    import sys
    code = ("import paper_2601_17561_amd, torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l or 'libhsa-runtime64' in l}\n"
            "print(len([x for x in libs if 'amdhip' in x]), len([x for x in libs if 'hsa-runtime' in x]))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout

