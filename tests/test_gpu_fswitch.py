"""GPU parity of FormatSwitch (Appendix C.1) against the oracle, element by element.

For each workload the library's key generation, transmission encryption and switch are compared with
oracle/formatswitch.py bit-exactly: the secrets s_T and s', every residue of the transmission
ciphertexts, and every residue of the switched query ciphertext.  The switched query then goes
through the CCMM in every form the shape allows and must decrypt to the popcount truth.
Workloads: 2^10 -> 2^7 (rho 8, two chunks per column, levels 2), 2^7 -> 2^7 (rho 1: the key switch
alone), 2^12 -> 2^9 (three chunks per column: two groups of conversion outputs), 2^15 -> 2^14 (the largest
query ring: two register groups per thread in the fused transforms), and the paper's
2^16 -> 2^13 at level 3 with 12,800-bit codes, checked against the oracle's hashes of every residue
(tests/golden/fs_paper.json, written by tests/golden/make_fs_paper.py from the oracle alone).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import hfe_synth as S

from oracle_cases import DB_SEED, KEY_SEED, TX_SEED, fs_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

FORMS = {"plain": H.HFE_FORM_PLAIN_U64, "i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(w, log_n_t, forms):
    """Library side: keys, FormatSwitch keys, transmission, switch, database; returns the pieces."""
    dev = torch.device("cuda", 0)
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    fk = H.hfe_fs_keygen(keys, w.level, log_n_t, KEY_SEED)
    inp = S.make_inputs(w)
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), torch.from_numpy(inp["q_masks"]).to(dev),
                       [int(s) for s in inp["shifts"]])
    T = H.hfe_fs_encrypt(fk, m_q, TX_SEED)
    qct = H.hfe_format_switch(fk, T, m_q.shape[0])
    m_db = H.hfe_encode(torch.from_numpy(inp["db_codes"]).to(dev), torch.from_numpy(inp["db_masks"]).to(dev), [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, sum(FORMS[f] for f in forms))
    torch.cuda.synchronize()
    return keys, fk, m_q, T, qct, db


def _forms(w):
    return [f for f in FORMS if f != "p2" or w.d2 + (1 << w.log_n_q) <= 1 << 16]


def _ccmm_decrypts_to_truth(w, db, qct, keys, ip_true, forms):
    for f in forms:
        r = H.hfe_ccmm(db, qct, 0, w.d1, FORMS[f])
        _, ip = H.hfe_decrypt(keys, r)
        torch.cuda.synchronize()
        assert np.array_equal(ip.cpu().numpy(), ip_true), f"{f}: decryption after FormatSwitch != popcount truth"


@pytest.mark.parametrize("wname", [S.FS_TINY.name, S.FS_FLAT.name, S.FS_MID.name, S.FS_WIDE.name])
def test_format_switch_bit_exact(wname):
    w = S.WORKLOADS[wname]
    _say(f"[gpu-fs] {wname}: oracle (CPU)")
    c = fs_case(wname)
    forms = _forms(w)
    _say(f"[gpu-fs] {wname}: library")
    keys, fk, m_q, T, qct, db = _run(w, c.log_n_t, forms)
    assert list(H.hfe_shape(fk)) == [w.level, c.log_n_t, c.F.rho, c.P.k]
    assert np.array_equal(m_q.cpu().numpy(), c.m_q)
    assert np.array_equal(H.hfe_export(fk, 0).view(np.int64), c.F.s_t)
    assert np.array_equal(H.hfe_export(fk, 1).view(np.int64), c.F.s_r)
    Tg = T.cpu().numpy().reshape(c.T.shape)
    for i in range(c.T.shape[0]):
        bad = np.argwhere(Tg[i] != c.T[i])
        assert bad.size == 0, f"transmission mod q_{i}: {len(bad)} residues differ, first {bad[:3].tolist()}"
    XT = H.hfe_export(qct, 0).reshape(c.XT.shape).astype(np.int64)
    for i in range(c.XT.shape[0]):
        bad = np.argwhere(XT[i] != c.XT[i])
        assert bad.size == 0, f"switched query mod q_{i}: {len(bad)} residues differ, first {bad[:3].tolist()}"
    _say(f"[gpu-fs] {wname}: CCMM ({', '.join(forms)})")
    _ccmm_decrypts_to_truth(w, db, qct, keys, c.ip_true, forms)


def _digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a.view(np.int64), dtype="<i8").tobytes()).hexdigest()


def _assert_matches(name, got: np.ndarray, g, what):
    assert int(np.prod(g["shapes"][name])) == got.size, f"{what}: {got.size} residues, oracle {g['shapes'][name]}"
    if _digest(got) == g["sha256"][name]:
        return
    msg = f"{what}: residues differ from the oracle"
    if name in g["samples"]:
        sm = g["samples"][name]
        flat = got.view(np.int64).reshape(-1)
        bad = [(i, int(flat[i]), v) for i, v in zip(sm["index"], sm["value"]) if int(flat[i]) != v]
        msg += f"; {len(bad)} of {len(sm['index'])} sampled entries differ, first {bad[:3]}"
    raise AssertionError(msg)


def test_format_switch_paper_degrees_match_the_oracle():
    w = S.FS_PAPER
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fs_paper.json")))[w.name]
    forms = _forms(w)
    _say(f"[gpu-fs] {w.name}: library ({', '.join(forms)})")
    keys, fk, m_q, T, qct, db = _run(w, g["log_n_t"], forms)
    _assert_matches("s_t", H.hfe_export(fk, 0), g, "s_T")
    _assert_matches("s_r", H.hfe_export(fk, 1), g, "s'")
    _assert_matches("T", T.cpu().numpy(), g, "transmission ciphertexts")
    _assert_matches("XT", H.hfe_export(qct, 0), g, "switched query")
    _ccmm_decrypts_to_truth(w, db, qct, keys, np.array(g["ip_true"]), forms)


def test_format_switch_profile_and_refusals():
    w = S.FS_TINY
    keys, fk, m_q, T, qct, db = _run(w, S.FS_LOG_N_T[w.name], ["plain"])
    H.hfe_profile(1)
    try:
        q2 = H.hfe_format_switch(fk, T, m_q.shape[0])
        ms = H.hfe_fs_profile_ms(q2, 4)
    finally:
        H.hfe_profile(0)
    assert all(x >= 0.0 for x in ms)
    assert np.array_equal(H.hfe_export(q2, 0), H.hfe_export(qct, 0))
    with pytest.raises(H.HfeError):
        H.hfe_fs_profile_ms(qct, 4)                               # made without profiling
    with pytest.raises(H.HfeError) as e:
        H.hfe_fs_keygen(keys, w.n_q_primes, 10, KEY_SEED)         # no prime left for the transmission
    assert e.value.status == -3
    for bad_log_n_t in (w.log_n_q - 1, 17):
        with pytest.raises(H.HfeError):
            H.hfe_fs_keygen(keys, w.level, bad_log_n_t, KEY_SEED)
    bad = torch.full((2, w.d2), 2, dtype=torch.int8, device="cuda")
    with pytest.raises(H.HfeError):
        H.hfe_fs_encrypt(fk, bad, TX_SEED)
    C = H.hfe_chain_default_params(9, 9, 7, 3, 512, 256)
    chain_keys = H.hfe_chain_keygen(C, KEY_SEED)
    with pytest.raises(H.HfeError):
        H.hfe_fs_keygen(chain_keys, 2, 10, KEY_SEED)
