"""Parity at one GPU's share of the paper's workload (N_DB = 2^14, N_Q = 2^13, 3 query primes
plus p, 14,336 database codes x 512 query columns of 12,800 bits), in the launch
configuration the benchmark times.

The oracle cannot materialise this size, so the checks are:
  * keys: every secret coefficient equals the oracle's;
  * database and query ciphertexts: sampled entries (A-part and B-part rows, every prime,
    first/last/ragged columns) and whole sampled query columns equal the oracle's
    single-entry evaluation of the same definitions;
  * CCMM result: sampled A-part entries recomputed by the oracle from its own database rows
    and query columns; the int8-MFMA result equals the plain result on every residue;
  * decryption: every one of the 7,340,032 inner products equals the brute-force popcount
    truth and lies within 0.25 of it; decisions and per-eye matches agree.
"""
import sys

import numpy as np
import pytest

import hfe_synth as S
from oracle import ckks as OC
from oracle import iris as OI
from oracle import params as OP
from oracle import prng

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

W = S.PAPER_SHARE
KEY_SEED, DB_SEED, Q_SEED = 41, 42, 43


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def run():
    w = W
    inp = S.make_inputs(w)
    dev = torch.device("cuda", 0)
    _say(f"[gpu-scale] {w.name}: keygen, encode, encrypt database")
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    db_codes = torch.from_numpy(inp["db_codes"]).to(dev)
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(s) for s in inp["shifts"]]
    m_db = H.hfe_encode(db_codes, db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED,
                          H.HFE_FORM_PLAIN_U64 | H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8)
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), q_masks, shifts)
    _say(f"[gpu-scale] {w.name}: encrypt query, ccmm i8 and plain")
    qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
    r_i8 = H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_I8_MFMA)
    r_pl = H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_PLAIN_U64)
    _say(f"[gpu-scale] {w.name}: ccmm rns")
    r_rns = H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_RNS_I8)
    _say(f"[gpu-scale] {w.name}: ccmm n^2")
    r_p2 = H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_P2_I8)
    _say(f"[gpu-scale] {w.name}: decrypt and match")
    v, ip = H.hfe_decrypt(keys, r_i8)
    dec, eye = H.hfe_match(ip, q_masks, shifts, db_masks)
    torch.cuda.synchronize()
    Po = OP.make_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys_o = OC.keygen(Po, KEY_SEED)
    from oracle import iris
    m_db_o = iris.ternary(inp["db_codes"], inp["db_masks"])
    qc, qm = iris.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    m_q_o = iris.ternary(qc, qm)
    return dict(inp=inp, keys=keys, db=db, qct=qct, r_i8=r_i8, r_pl=r_pl, r_rns=r_rns, r_p2=r_p2, v=v, ip=ip, dec=dec, eye=eye,
                Po=Po, keys_o=keys_o, m_db_o=m_db_o, m_q_o=m_q_o, qc=qc, qm=qm, m_q=m_q)


def test_encoding_and_keys(run):
    assert np.array_equal(run["m_q"].cpu().numpy(), run["m_q_o"])
    ko = run["keys_o"]
    s = H.hfe_export(run["keys"], 0).view(np.int64).reshape(ko.s.shape)
    sdb = H.hfe_export(run["keys"], 1).view(np.int64).reshape(ko.s_db.shape)
    assert np.array_equal(s, ko.s) and np.array_equal(sdb, ko.s_db)


def test_db_sampled_entries(run):
    Po, ko = run["Po"], run["keys_o"]
    R = Po.n_db + W.d1
    rng = np.random.default_rng(1)
    cols = [0, Po.d2 - 1, Po.d2, Po.K - 1] + rng.integers(0, Po.K, 4).tolist()
    rows = [0, Po.n_db - 1, Po.n_db, R - 1] + rng.integers(0, R, 4).tolist()
    ids = OC.prime_ids(Po, len(Po.q))
    for z, (pid, prime) in enumerate(ids):
        for r, c in zip(rows, cols):
            got = int(H.hfe_export(run["db"], 0, (z * Po.K + c) * R + r, 1)[0])
            exp = OC.db_entry(ko, run["m_db_o"], DB_SEED, pid, prime, r, c)
            assert got == exp, (z, r, c)


_qcols = {}


def _query_col(run, c):
    if c not in _qcols:
        _qcols[c] = OC.query_column(run["keys_o"], run["m_q_o"][c], W.level, Q_SEED, c)
    return _qcols[c]


def test_query_sampled_columns(run):
    K = run["Po"].K
    for c in (0, 77, W.d3 - 1):
        exp = _query_col(run, c)
        for i in range(W.level):
            got = H.hfe_export(run["qct"], 0, (i * W.d3 + c) * K, K).astype(np.int64)
            assert np.array_equal(got, exp[i]), (i, c)


def test_ccmm_sampled_a_part_entries(run):
    Po = run["Po"]
    R_out = Po.n_db + W.d1
    ids = OC.prime_ids(Po, W.level)
    kk = np.arange(Po.K)
    for r, c in ((0, 0), (Po.n_db - 1, 77), (5000, W.d3 - 1)):
        d_row = {pid: prng.uniform_mod(DB_SEED, prng.DBA, pid, np.full(Po.K, r), kk, prime) for pid, prime in ids}
        exp = OC.ccmm_entry(Po, d_row, _query_col(run, c), W.level)
        for name in ("r_i8", "r_pl", "r_rns", "r_p2"):
            for i in range(W.level):
                got = int(H.hfe_export(run[name], 0, (i * W.d3 + c) * R_out + r, 1)[0])
                assert got == exp[i], (name, i, r, c)


def test_i8_equals_plain_on_every_residue(run):
    a = H.hfe_export(run["r_i8"], 0)
    b = H.hfe_export(run["r_pl"], 0)
    assert a.shape == b.shape and np.array_equal(a, b)


def test_rns_equals_i8_on_every_residue(run):
    a = H.hfe_export(run["r_rns"], 0)
    b = H.hfe_export(run["r_i8"], 0)
    assert a.shape == b.shape and np.array_equal(a, b)


def test_n2_form_equals_i8_on_every_residue(run):
    a = H.hfe_export(run["r_p2"], 0)
    b = H.hfe_export(run["r_i8"], 0)
    assert a.shape == b.shape and np.array_equal(a, b)


def test_decrypt_equals_popcount_truth_on_all_pairs(run):
    inp = run["inp"]
    ip_true, ov = OI.truth(run["qc"], run["qm"], inp["db_codes"], inp["db_masks"])
    ip = run["ip"].cpu().numpy()
    v = run["v"].cpu().numpy()
    assert ip.shape == (W.d3, W.d1)
    assert np.array_equal(ip, ip_true)
    assert np.abs(v - ip_true).max() <= 0.25
    dec_ref = OI.decide(ip_true, ov)
    assert np.array_equal(run["dec"].cpu().numpy().astype(bool), dec_ref)
    eye_ref = OI.match_per_eye(dec_ref, W.n_shifts)
    assert np.array_equal(run["eye"].cpu().numpy().astype(bool), eye_ref)
    assert eye_ref.sum() >= len(S.planted_for(W))      # planted eyes are found
    _say(f"[gpu-scale] max |v - IP| = {np.abs(v - ip_true).max():.4f}, matches {int(dec_ref.sum())}")
