"""GPU parity of the CCMM over the paper's n^2 modulus chain (Section 6.3) against the chain oracle.

Keys from hfe_chain_keygen (7 query moduli n^2 and 3 special moduli, the largest primes of
[127, 253]); element by element against oracle/chain.py, bit-exact: the secrets, every residue of the
database (each modulus n^2), of the query and of the CCMM result, at the full level and at a lower one;
decryption equals the oracle's and the popcount truth.  The tiny workload has rings of 2^9; the mid
workload's shapes cross every tile boundary of the n^2 contraction (956 output rows, 272 columns); a
row shard equals the full result restricted to its rows.  Calls outside the chain's scope are refused.
"""
import sys

import numpy as np
import pytest

import hfe_synth as S

from oracle_cases import CHAIN_P_MODS, DB_SEED, KEY_SEED, Q_SEED, chain_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(w, level):
    dev = torch.device("cuda", 0)
    C = H.hfe_chain_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, CHAIN_P_MODS, w.d2, w.d1)
    keys = H.hfe_chain_keygen(C, KEY_SEED)
    inp = S.make_inputs(w)
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(x) for x in inp["shifts"]]
    m_db = H.hfe_encode(torch.from_numpy(inp["db_codes"]).to(dev), db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, H.HFE_FORM_P2_I8 | H.HFE_FORM_PLAIN_U64)
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), q_masks, shifts)
    qct = H.hfe_encrypt(keys, m_q, level, Q_SEED)
    torch.cuda.synchronize()
    return C, keys, db, qct


def _check_all(w, level):
    c = chain_case(w.name, level)
    C, keys, db, qct = _setup(w, level)
    assert C.q_bases() == list(c.C.q_bases) and C.p_bases() == list(c.C.p_bases)
    assert np.array_equal(H.hfe_export(keys, 0).view(np.int64).reshape(c.keys.s.shape), c.keys.s)
    assert np.array_equal(H.hfe_export(keys, 1).view(np.int64).reshape(c.keys.s_db.shape), c.keys.s_db)
    bases = c.C.all_bases()
    D = H.hfe_export(db, 0).reshape(len(bases), c.C.K, -1).astype(np.int64)
    for i, n in enumerate(bases):
        bad = np.argwhere(D[i] != c.D[n].T)
        assert bad.size == 0, f"database mod {n}^2: {len(bad)} residues differ, first {bad[:3].tolist()}"
    XT = H.hfe_export(qct, 0).reshape(level, c.m_q.shape[0], -1).astype(np.int64)
    for j, n in enumerate(c.C.q_bases[:level]):
        assert np.array_equal(XT[j], c.XT[n]), f"query mod {n}^2 differs"
    r = H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_P2_I8)
    out = H.hfe_export(r, 0).reshape(level, c.m_q.shape[0], -1).astype(np.int64)
    for j, n in enumerate(c.C.q_bases[:level]):
        bad = np.argwhere(out[j] != c.out[n])
        assert bad.size == 0, f"result mod {n}^2: {len(bad)} residues differ, first {bad[:3].tolist()}"
    v, ip = H.hfe_decrypt(keys, r)
    torch.cuda.synchronize()
    assert np.array_equal(ip.cpu().numpy(), c.ip)
    assert np.array_equal(c.ip, c.ip_true)
    err = float(np.max(np.abs(v.cpu().numpy() - c.ip_true)))
    assert err <= 0.25
    return c, keys, db, qct, out


@pytest.mark.parametrize("level", [7, 5])
def test_chain_tiny_bit_exact(level):
    _say(f"[gpu-chain] {S.CHAIN_TINY.name} level {level}")
    _check_all(S.CHAIN_TINY, level)


def test_chain_mid_bit_exact_and_row_shard():
    w = S.CHAIN_MID
    _say(f"[gpu-chain] {w.name}: oracle (CPU) and GPU")
    c, keys, db, qct, out = _check_all(w, w.n_q_primes)
    row0, rows = 150, 431
    r = H.hfe_ccmm(db, qct, row0, rows, H.HFE_FORM_P2_I8)
    sh = H.hfe_export(r, 0).reshape(w.n_q_primes, c.m_q.shape[0], -1).astype(np.int64)
    n_db = 1 << w.log_n_db
    exp = np.concatenate([out[:, :, :n_db], out[:, :, n_db + row0:n_db + row0 + rows]], axis=2)
    assert np.array_equal(sh, exp)
    _, ip = H.hfe_decrypt(keys, r)
    torch.cuda.synchronize()
    assert np.array_equal(ip.cpu().numpy(), c.ip_true[:, row0:row0 + rows])


def test_chain_noalloc_equals_single_call():
    w = S.CHAIN_TINY
    C, keys, db, qct = _setup(w, w.n_q_primes)
    ref = H.hfe_export(H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_P2_I8), 0).astype(np.int64)
    out = torch.full((w.n_q_primes, w.d3, (1 << w.log_n_db) + w.d1), -1, dtype=torch.int64, device="cuda")
    H.hfe_ccmm_noalloc(db, qct, 0, w.d1, H.HFE_FORM_P2_I8, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1), ref)


def test_chain_refusals():
    w = S.CHAIN_TINY
    C, keys, db, qct = _setup(w, w.n_q_primes)
    for form in (H.HFE_FORM_I8_MFMA, H.HFE_FORM_PLAIN_U64):
        with pytest.raises(H.HfeError):
            H.hfe_ccmm(db, qct, 0, w.d1, form)
    with pytest.raises(H.HfeError):
        H.hfe_ccmm_batched(db, [(qct, 0, w.d1)], H.HFE_FORM_P2_I8)
    with pytest.raises(H.HfeError):
        H.hfe_plan_create(db, 4, 64, 2, H.HFE_FORM_P2_I8)
    with pytest.raises(H.HfeError) as e:
        H.hfe_encrypt(keys, torch.zeros((2, w.d2), dtype=torch.int8, device="cuda"), 8, Q_SEED)
    assert e.value.status == -3
    bad = H.hfe_chain_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, CHAIN_P_MODS, w.d2, w.d1)
    bad.bases[1] = bad.bases[0]
    with pytest.raises(H.HfeError):
        H.hfe_chain_keygen(bad, 1)
