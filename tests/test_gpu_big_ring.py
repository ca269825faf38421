"""GPU parity at ring degree 2^16 (two-pass transforms through device memory).

Two workloads, each with one layer at 2^16 so that the full-matrix oracle stays tractable:
BIG_DB (N_DB = 2^16, N_Q = 2^9: the database secret products of encryption and decryption at
2^16) and BIG_Q (N_DB = 2^9, N_Q = 2^16: the query secret products of query encryption and of
T = M_DB S_Q at 2^16).  tests/golden/big_ring.json holds the oracle's SHA-256 of every residue array
(keys, database, query, CCMM result) in the library's export order, written by
tests/golden/make_big_ring.py from the oracle alone; equal hashes mean every residue is equal.
The CCMM runs in every form the shape allows (the n^2 form needs K <= 2^16, so BIG_Q skips it) and
must decrypt to the oracle's inner products, which equal the popcount truth.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import hfe_synth as S
from oracle import iris as OI

from oracle_cases import DB_SEED, KEY_SEED, Q_SEED

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "big_ring.json")))
FORMS = {"plain": H.HFE_FORM_PLAIN_U64, "i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a.view(np.int64), dtype="<i8").tobytes()).hexdigest()


def _assert_matches(name, got: np.ndarray, g, what):
    exp_shape = g["shapes"][name]
    assert int(np.prod(exp_shape)) == got.size, f"{what}: {got.size} residues, oracle {exp_shape}"
    if _digest(got) == g["sha256"][name]:
        return
    msg = f"{what}: residues differ from the oracle"
    if name in g["samples"]:
        sm = g["samples"][name]
        flat = got.view(np.int64).reshape(-1)
        bad = [(i, int(flat[i]), v) for i, v in zip(sm["index"], sm["value"]) if int(flat[i]) != v]
        msg += f"; {len(bad)} of {len(sm['index'])} sampled entries differ, first {bad[:3]}"
    raise AssertionError(msg)


@pytest.mark.parametrize("wname", [S.BIG_DB.name, S.BIG_Q.name])
def test_ring_degree_2_16_matches_the_oracle(wname):
    w = S.WORKLOADS[wname]
    g = GOLDEN[w.name]
    dev = torch.device("cuda", 0)
    K = w.d2 + (1 << w.log_n_q)
    forms = [f for f in FORMS if f != "p2" or K <= 1 << 16]
    _say(f"[gpu-big] {w.name}: keygen")
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    _assert_matches("s_q", H.hfe_export(keys, 0), g, "query secrets")
    _assert_matches("s_db", H.hfe_export(keys, 1), g, "database secrets")
    inp = S.make_inputs(w)
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(s) for s in inp["shifts"]]
    _say(f"[gpu-big] {w.name}: database encryption ({', '.join(forms)})")
    m_db = H.hfe_encode(torch.from_numpy(inp["db_codes"]).to(dev), db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, sum(FORMS[f] for f in forms))
    torch.cuda.synchronize()
    _assert_matches("D", H.hfe_export(db, 0), g, "database D")
    _say(f"[gpu-big] {w.name}: query encryption")
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), q_masks, shifts)
    qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
    _assert_matches("XT", H.hfe_export(qct, 0), g, "query ciphertext")
    qc, qm = OI.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    ip_true, _ = OI.truth(qc, qm, inp["db_codes"], inp["db_masks"])
    ip_oracle = np.array(g["ip"], dtype=np.int64)
    assert np.array_equal(ip_oracle, ip_true)
    for f in forms:
        _say(f"[gpu-big] {w.name}: CCMM, form {f}")
        r = H.hfe_ccmm(db, qct, 0, w.d1, FORMS[f])
        _assert_matches("out", H.hfe_export(r, 0), g, f"result ({f})")
        _, ip = H.hfe_decrypt(keys, r)
        torch.cuda.synchronize()
        assert np.array_equal(ip.cpu().numpy(), ip_oracle), f"{f}: decrypted inner products differ"
