"""GPU parity of the HIP library against the CPU oracle (bit-exact residues).

For each small workload the whole hot path runs through the C ABI on the GPU: masked ternary
encoding, key generation, database and query encryption, the CCMM in both forms (plain
uint64 and int8 MFMA), rescale, decryption and the match decision.  Every residue of every
handle is compared with the oracle element by element; decrypted inner products must equal
the brute-force popcount truth and lie within 0.25 of it; decisions must agree.
"""
import sys

import numpy as np
import pytest

import hfe_synth as S
from oracle import ckks as OC
from oracle import iris as OI

from oracle_cases import DB_SEED, KEY_SEED, Q_SEED, case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

FORMS = {"plain": H.HFE_FORM_PLAIN_U64, "i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class GpuRun:
    """The hot path of one oracle case on the GPU."""

    def __init__(self, c, forms=H.HFE_FORM_PLAIN_U64 | H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8):
        w = c.w
        _say(f"[gpu] {w.name}: keygen / encode / encrypt_db")
        self.c = c
        self.P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
        self.keys = H.hfe_keygen(self.P, KEY_SEED)
        inp = c.inputs
        self.db_codes = torch.from_numpy(inp["db_codes"]).cuda()
        self.db_masks = torch.from_numpy(inp["db_masks"]).cuda()
        self.q_codes = torch.from_numpy(inp["q_codes"]).cuda()
        self.q_masks = torch.from_numpy(inp["q_masks"]).cuda()
        self.shifts = [int(s) for s in inp["shifts"]]
        self.m_db = H.hfe_encode(self.db_codes, self.db_masks, [0])
        self.db = H.hfe_encrypt_db(self.keys, self.m_db, DB_SEED, forms)
        _say(f"[gpu] {w.name}: encode / encrypt query")
        self.m_q = H.hfe_encode(self.q_codes, self.q_masks, self.shifts)
        self.qct = H.hfe_encrypt(self.keys, self.m_q, w.level, Q_SEED)
        torch.cuda.synchronize()

    def ccmm(self, form, row0=None, rows=None):
        c = self.c
        row0 = c.row0 if row0 is None else row0
        rows = c.rows if rows is None else rows
        _say(f"[gpu] {c.w.name}: ccmm form={form} rows=[{row0}, {row0 + rows})")
        r = H.hfe_ccmm(self.db, self.qct, row0, rows, FORMS[form])
        torch.cuda.synchronize()
        return r


_runs = {}


def run_for(name, row0=0, rows=-1):
    key = (name, row0, rows)
    if key not in _runs:
        _runs[key] = GpuRun(case(name, row0, rows))
    return _runs[key]


CASES = [(S.TINY.name, 0, -1), (S.TINY_MULTI.name, 0, -1), (S.TINY_MULTI.name, 100, 60)]
IDS = ["tiny", "tinymulti", "tinymulti_shard"]


@pytest.mark.parametrize("name,row0,rows", CASES, ids=IDS)
def test_encode_matches_oracle(name, row0, rows):
    g = run_for(name, row0, rows)
    c = g.c
    assert np.array_equal(g.m_db.cpu().numpy(), c.m_db)
    assert np.array_equal(g.m_q.cpu().numpy(), c.m_q)


@pytest.mark.parametrize("name,row0,rows", CASES[:2], ids=IDS[:2])
def test_keys_match_oracle(name, row0, rows):
    g = run_for(name, row0, rows)
    s = H.hfe_export(g.keys, 0).view(np.int64).reshape(g.c.keys.s.shape)
    sdb = H.hfe_export(g.keys, 1).view(np.int64).reshape(g.c.keys.s_db.shape)
    assert np.array_equal(s, g.c.keys.s) and np.array_equal(sdb, g.c.keys.s_db)


@pytest.mark.parametrize("name,row0,rows", CASES[:2], ids=IDS[:2])
def test_db_ciphertext_bit_exact(name, row0, rows):
    g = run_for(name, row0, rows)
    c = g.c
    P = c.P
    D = H.hfe_export(g.db, 0).reshape(len(P.q) + 1, P.K, P.n_db + c.w.d1).astype(np.int64)
    for z, (pid, _) in enumerate(OC.prime_ids(P, len(P.q))):
        bad = np.argwhere(D[z].T != c.D[pid])
        assert bad.size == 0, f"prime slot {z}: {len(bad)} mismatches, first {bad[:3].tolist()}"


@pytest.mark.parametrize("name,row0,rows", CASES[:2], ids=IDS[:2])
def test_query_ciphertext_bit_exact(name, row0, rows):
    g = run_for(name, row0, rows)
    c = g.c
    XT = H.hfe_export(g.qct, 0).reshape(c.w.level, c.m_q.shape[0], c.P.K).astype(np.int64)
    for i in range(c.w.level):
        assert np.array_equal(XT[i], c.XT[i]), f"prime {i}"


@pytest.mark.parametrize("form", ["plain", "i8", "rns", "p2"])
@pytest.mark.parametrize("name,row0,rows", CASES, ids=IDS)
def test_ccmm_result_bit_exact(name, row0, rows, form):
    g = run_for(name, row0, rows)
    c = g.c
    r = g.ccmm(form)
    out = H.hfe_export(r, 0).reshape(c.w.level, c.m_q.shape[0], c.P.n_db + c.rows).astype(np.int64)
    for i in range(c.w.level):
        bad = np.argwhere(out[i] != c.out[i])
        assert bad.size == 0, f"{form} prime {i}: {len(bad)} mismatches, first {bad[:3].tolist()}"


@pytest.mark.parametrize("name,row0,rows", CASES, ids=IDS)
def test_every_i8_tile_configuration_bit_exact(name, row0, rows):
    """Each int8 tile configuration (register-staged, pipelined, LDS-DMA) gives the oracle's residues."""
    g = run_for(name, row0, rows)
    c = g.c
    try:
        for v in range(H.hfe_i8_variants()):
            H.hfe_set_i8_variant(v)
            _say(f"[gpu] {c.w.name}: ccmm i8 tile {H.hfe_i8_variant_name(v)}")
            r = g.ccmm("i8")
            out = H.hfe_export(r, 0).reshape(c.w.level, c.m_q.shape[0], c.P.n_db + c.rows).astype(np.int64)
            for i in range(c.w.level):
                bad = np.argwhere(out[i] != c.out[i])
                assert bad.size == 0, f"{H.hfe_i8_variant_name(v)} prime {i}: {len(bad)} mismatches"
    finally:
        H.hfe_set_i8_variant(-1)


@pytest.mark.parametrize("form", ["plain", "i8", "rns", "p2"])
@pytest.mark.parametrize("name,row0,rows", CASES, ids=IDS)
def test_decrypt_and_match_equal_popcount_truth(name, row0, rows, form):
    g = run_for(name, row0, rows)
    c = g.c
    r = g.ccmm(form)
    _say(f"[gpu] {c.w.name}: decrypt / match")
    v, ip = H.hfe_decrypt(g.keys, r)
    dec, eye = H.hfe_match(ip, g.q_masks, g.shifts, g.db_masks[c.row0:c.row0 + c.rows].contiguous())
    torch.cuda.synchronize()
    ip = ip.cpu().numpy()
    v = v.cpu().numpy()
    assert np.array_equal(ip, c.ip) and np.array_equal(ip, c.ip_true)
    assert np.abs(v - c.ip_true).max() <= 0.25
    vo = np.array([[float(x) for x in row] for row in c.v])
    assert np.abs(v - vo).max() < 1e-9
    dec_ref = OI.decide(c.ip_true, c.overlap)
    assert np.array_equal(dec.cpu().numpy().astype(bool), dec_ref)
    assert np.array_equal(eye.cpu().numpy().astype(bool), OI.match_per_eye(dec_ref, c.w.n_shifts))


def test_level_below_database_primes():
    """A level-1 query against a database carrying two query primes (subset of its primes)."""
    c = case(S.TINY_MULTI.name)
    g = run_for(S.TINY_MULTI.name)
    XT = OC.encrypt_query(c.keys, c.m_q, 1, Q_SEED + 7)
    out = OC.ccmm(c.P, c.D, XT, 1, 0, c.w.d1)
    _, ip_o = OC.decrypt(c.keys, out, 1, 0, c.w.d1)
    _say("[gpu] tinymulti: level-1 query")
    qct = H.hfe_encrypt(g.keys, g.m_q, 1, Q_SEED + 7)
    for form in ("plain", "i8", "rns", "p2"):
        r = H.hfe_ccmm(g.db, qct, 0, c.w.d1, FORMS[form])
        got = H.hfe_export(r, 0).reshape(1, c.m_q.shape[0], -1).astype(np.int64)
        assert np.array_equal(got[0], out[0]), form
        _, ip = H.hfe_decrypt(g.keys, r)
        assert np.array_equal(ip.cpu().numpy(), ip_o)
        assert np.array_equal(ip_o, c.ip_true)


def test_api_errors_on_device_handles():
    g = run_for(S.TINY_MULTI.name)
    with pytest.raises(H.HfeError) as e:
        H.hfe_ccmm(g.db, g.qct, 200, 100, H.HFE_FORM_I8_MFMA)        # rows beyond d1
    assert e.value.status == -2
    with pytest.raises(H.HfeError) as e:
        H.hfe_ccmm(g.db, g.qct, 0, 10, 3)                            # unknown form
    assert e.value.status == -1
    with pytest.raises(H.HfeError) as e:
        H.hfe_encrypt(g.keys, g.m_q, 3, 1)                          # level above L = 2
    assert e.value.status == -3
