"""Saving and loading the encrypted database (hfe_db_save / hfe_db_load).

A database written to a file and read back under the same keys must give bit-identical results in
every form it was prepared for (and the same plain residues), also when only some of its forms are
loaded; a file written under other keys, a truncated file, a file with trailing bytes, a file that
is not a database and a request for a form the file lacks are refused.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

ALL = H.HFE_FORM_PLAIN_U64 | H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8
INT8 = (H.HFE_FORM_I8_MFMA, H.HFE_FORM_RNS_I8, H.HFE_FORM_P2_I8)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    log_n_db, log_n_q, d1, d2, level, d3 = 8, 9, 150, 700, 2, 7
    dev = torch.device("cuda", 0)
    P = H.hfe_default_params(log_n_db, log_n_q, level, d2, d1)
    keys = H.hfe_keygen(P, 61)
    other = H.hfe_keygen(P, 62)
    rng = np.random.default_rng(63)
    m_db = torch.from_numpy(rng.integers(-1, 2, (d1, d2)).astype(np.int8)).to(dev)
    m_q = torch.from_numpy(rng.integers(-1, 2, (d3, d2)).astype(np.int8)).to(dev)
    _say("[gpu-store] keygen, encrypt the database in every form")
    db = H.hfe_encrypt_db(keys, m_db, 64, ALL)
    q = H.hfe_encrypt(keys, m_q, level, 65)
    torch.cuda.synchronize()
    return dict(keys=keys, other=other, db=db, q=q, d1=d1)


def _result(db, q, row0, rows, form):
    return H.hfe_export(H.hfe_ccmm(db, q, row0, rows, form), 0)


def test_round_trip_gives_identical_results_in_every_form(env, tmp_path):
    path = tmp_path / "db.hfe"
    _say("[gpu-store] save, load")
    H.hfe_db_save(env["db"], path)
    loaded = H.hfe_db_load(env["keys"], path)
    assert np.array_equal(H.hfe_export(loaded, 0), H.hfe_export(env["db"], 0))
    for form in (H.HFE_FORM_PLAIN_U64,) + INT8:
        for row0, rows in ((0, env["d1"]), (37, 50)):
            _say(f"[gpu-store] ccmm form {form} rows [{row0}, {row0 + rows})")
            a = _result(env["db"], env["q"], row0, rows, form)
            b = _result(loaded, env["q"], row0, rows, form)
            assert np.array_equal(a, b), f"form {form}: loaded database differs"


def test_subset_of_forms_round_trips(env, tmp_path):
    m_db = torch.from_numpy(np.random.default_rng(66).integers(-1, 2, (40, 700)).astype(np.int8)).cuda()
    db = H.hfe_encrypt_db(env["keys"], m_db, 67, H.HFE_FORM_RNS_I8)
    path = tmp_path / "rns.hfe"
    H.hfe_db_save(db, path)
    loaded = H.hfe_db_load(env["keys"], path)
    assert np.array_equal(_result(db, env["q"], 0, 40, H.HFE_FORM_RNS_I8),
                          _result(loaded, env["q"], 0, 40, H.HFE_FORM_RNS_I8))
    with pytest.raises(H.HfeError) as e:                            # not prepared for the digit form
        H.hfe_ccmm(loaded, env["q"], 0, 40, H.HFE_FORM_I8_MFMA)
    assert e.value.status == -1


def test_loading_a_subset_of_the_stored_forms(env, tmp_path):
    path = tmp_path / "all.hfe"
    H.hfe_db_save(env["db"], path)
    d1 = env["d1"]
    for form in INT8:
        _say(f"[gpu-store] load only form {form}")
        one = H.hfe_db_load(env["keys"], path, form)
        assert np.array_equal(_result(one, env["q"], 0, d1, form), _result(env["db"], env["q"], 0, d1, form))
        other = H.HFE_FORM_PLAIN_U64 if form != H.HFE_FORM_PLAIN_U64 else H.HFE_FORM_I8_MFMA
        with pytest.raises(H.HfeError) as e:                        # the skipped forms are absent
            H.hfe_ccmm(one, env["q"], 0, d1, other)
        assert e.value.status == -1
        one.free()
    m_db = torch.from_numpy(np.random.default_rng(68).integers(-1, 2, (20, 700)).astype(np.int8)).cuda()
    rns_only = tmp_path / "rns_only.hfe"
    H.hfe_db_save(H.hfe_encrypt_db(env["keys"], m_db, 69, H.HFE_FORM_RNS_I8), rns_only)
    with pytest.raises(H.HfeError) as e:                            # a form the file lacks
        H.hfe_db_load(env["keys"], rns_only, H.HFE_FORM_P2_I8)
    assert e.value.status == -1 and "requested form" in str(e.value)


def test_database_bytes_follow_the_storage_formula(env, tmp_path):
    """Section 6.3's storage count: (N_DB + d1)(d2 + N_Q) entries per prime, times 8 / 5 / n / 2n bytes for
    the four forms, in the padded plane layout (K up to a multiple of 64, rows up to a multiple of 64
    plus 256 zero rows), and the same size a saved file carries."""
    log_n_db, log_n_q, d1, d2, level = 8, 9, 150, 700, 2
    R, K, primes = (1 << log_n_db) + d1, d2 + (1 << log_n_q), level + 1
    KB, R_pad = (K + 63) // 64, (R + 63) // 64 * 64 + 256
    db = env["db"]
    plain = H.hfe_db_bytes(db, H.HFE_FORM_PLAIN_U64)
    assert plain == R * K * primes * 8                                    # exactly the formula
    digits = H.hfe_db_bytes(db, H.HFE_FORM_I8_MFMA)
    assert digits == primes * 5 * KB * R_pad * 64 and digits >= R * K * primes * 5
    rns, p2 = H.hfe_db_bytes(db, H.HFE_FORM_RNS_I8), H.hfe_db_bytes(db, H.HFE_FORM_P2_I8)
    plane = primes * KB * R_pad * 64
    assert rns % plane == 0 and p2 % (2 * plane) == 0                     # n moduli, n bases (2 planes each)
    n_rns, n_p2 = rns // plane, p2 // (2 * plane)
    assert 1 <= n_rns <= 16 and 1 <= n_p2 <= 8
    assert H.hfe_db_bytes(db) == plain + digits + rns + p2
    path = tmp_path / "size.hfe"
    H.hfe_db_save(db, path)
    assert path.stat().st_size == 104 + H.hfe_db_bytes(db)               # header + every form's planes
    with pytest.raises(H.HfeError):
        H.hfe_db_bytes(db, 3)                                             # not one form


def test_bad_files_are_refused(env, tmp_path):
    path = tmp_path / "db.hfe"
    H.hfe_db_save(env["db"], path)
    data = path.read_bytes()
    with pytest.raises(H.HfeError) as e:                            # other keys
        H.hfe_db_load(env["other"], path)
    assert e.value.status == -1 and "other keys" in str(e.value)
    short = tmp_path / "short.hfe"
    short.write_bytes(data[:-1000])
    with pytest.raises(H.HfeError) as e:
        H.hfe_db_load(env["keys"], short)
    assert e.value.status == -1 and "truncated" in str(e.value)
    longer = tmp_path / "long.hfe"
    longer.write_bytes(data + b"\0")
    with pytest.raises(H.HfeError) as e:
        H.hfe_db_load(env["keys"], longer)
    assert e.value.status == -1 and "trailing" in str(e.value)
    junk = tmp_path / "junk.hfe"
    junk.write_bytes(os.urandom(4096))
    with pytest.raises(H.HfeError) as e:
        H.hfe_db_load(env["keys"], junk)
    assert e.value.status == -1
    with pytest.raises(H.HfeError) as e:
        H.hfe_db_load(env["keys"], tmp_path / "missing.hfe")
    assert e.value.status == -1
