"""GPU parity on the mid-size workload, element by element against the CPU oracle.

The workload's shapes cross every tile boundary of the contraction kernels: 956 output rows
(256 A-part rows and 700 database codes: ragged against 64-, 128- and 256-row tiles), 272 query
columns (17 eyes x 16 shifts: two 128-column tiles plus 16, one 256-column tile plus 16),
K = 1,280 + 512 = 1,792 (28 blocks of 64), three query primes plus p, and three secrets per
stack (the last chunk truncated).  Every residue of the database, the query, the exact product
before the rescale and the result is compared with the oracle in all four forms and every digit
tile configuration, on the full row range and a row shard; batches (one persistent launch) and a
plan replayed through its captured hipGraph are compared the same way; decryption and decisions
equal the popcount truth.

The oracle of a row shard is the full oracle result restricted to the A-part rows and the shard's
codes (rows are independent; pinned on the CPU by test_ccmm_on_a_row_shard_matches_the_full_result).
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
W = S.MID
SHARD = (150, 431)          # codes [150, 581): B rows start and end inside row tiles


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mid():
    _say(f"[gpu-mid] {W.name}: oracle (CPU)")
    c = case(W.name)
    pre = OC.ccmm_pre_rescale(c.P, c.D, c.XT, W.level, 0, W.d1)
    dev = torch.device("cuda", 0)
    _say(f"[gpu-mid] {W.name}: keygen, encrypt database and query")
    P = H.hfe_default_params(W.log_n_db, W.log_n_q, W.n_q_primes, W.d2, W.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    inp = c.inputs
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(s) for s in inp["shifts"]]
    m_db = H.hfe_encode(torch.from_numpy(inp["db_codes"]).to(dev), db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, sum(FORMS.values()))
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), q_masks, shifts)
    qct = H.hfe_encrypt(keys, m_q, W.level, Q_SEED)
    torch.cuda.synchronize()
    return dict(c=c, pre=pre, keys=keys, db=db, qct=qct, m_db=m_db, m_q=m_q, db_masks=db_masks, q_masks=q_masks,
                shifts=shifts)


def _expected(c, row0, rows):
    """Oracle result residues [prime][column][A rows | codes row0 .. row0 + rows)."""
    n = c.P.n_db
    return np.stack([np.concatenate([c.out[i][:, :n], c.out[i][:, n + row0:n + row0 + rows]], axis=1)
                     for i in range(W.level)])


def _result(r, rows):
    return H.hfe_export(r, 0).reshape(W.level, W.d3, -1).astype(np.int64)


def _assert_equal(got, exp, what):
    bad = np.argwhere(got != exp)
    assert bad.size == 0, f"{what}: {len(bad)} mismatches, first {bad[:3].tolist()}"


def test_mid_ciphertexts_bit_exact(mid):
    c = mid["c"]
    assert np.array_equal(mid["m_db"].cpu().numpy(), c.m_db)
    assert np.array_equal(mid["m_q"].cpu().numpy(), c.m_q)
    P = c.P
    D = H.hfe_export(mid["db"], 0).reshape(len(P.q) + 1, P.K, P.n_db + W.d1).astype(np.int64)
    for z, (pid, _) in enumerate(OC.prime_ids(P, len(P.q))):
        _assert_equal(D[z].T, c.D[pid], f"database prime slot {z}")
    XT = H.hfe_export(mid["qct"], 0).reshape(W.level, W.d3, P.K).astype(np.int64)
    for i in range(W.level):
        _assert_equal(XT[i], c.XT[i], f"query prime {i}")


@pytest.mark.parametrize("form", list(FORMS))
def test_mid_product_before_rescale_bit_exact(mid, form):
    c = mid["c"]
    _say(f"[gpu-mid] product before rescale, form {form}")
    C = H.hfe_ccmm_product(mid["db"], mid["qct"], 0, W.d1, FORMS[form]).cpu().numpy()
    for z, (pid, _) in enumerate(OC.prime_ids(c.P, W.level)):
        _assert_equal(C[z], mid["pre"][pid].T, f"{form} product, prime slot {z}")


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("row0,rows", [(0, W.d1), SHARD], ids=["full", "shard"])
def test_mid_result_bit_exact(mid, form, row0, rows):
    _say(f"[gpu-mid] ccmm form {form} rows [{row0}, {row0 + rows})")
    r = H.hfe_ccmm(mid["db"], mid["qct"], row0, rows, FORMS[form])
    _assert_equal(_result(r, rows), _expected(mid["c"], row0, rows), f"{form} result")


@pytest.mark.parametrize("row0,rows", [(0, W.d1), SHARD], ids=["full", "shard"])
def test_mid_every_digit_tile_bit_exact(mid, row0, rows):
    exp = _expected(mid["c"], row0, rows)
    try:
        for v in range(H.hfe_i8_variants()):
            H.hfe_set_i8_variant(v)
            _say(f"[gpu-mid] digit tile {H.hfe_i8_variant_name(v)} rows [{row0}, {row0 + rows})")
            r = H.hfe_ccmm(mid["db"], mid["qct"], row0, rows, H.HFE_FORM_I8_MFMA)
            _assert_equal(_result(r, rows), exp, f"tile {H.hfe_i8_variant_name(v)}")
    finally:
        H.hfe_set_i8_variant(-1)


def test_mid_decrypt_and_match_equal_popcount_truth(mid):
    c = mid["c"]
    for form in FORMS:
        r = H.hfe_ccmm(mid["db"], mid["qct"], 0, W.d1, FORMS[form])
        v, ip = H.hfe_decrypt(mid["keys"], r)
        dec, eye = H.hfe_match(ip, mid["q_masks"], mid["shifts"], mid["db_masks"])
        torch.cuda.synchronize()
        ip = ip.cpu().numpy()
        assert np.array_equal(ip, c.ip_true), form
        assert np.abs(v.cpu().numpy() - c.ip_true).max() <= 0.25
        dec_ref = OI.decide(c.ip_true, c.overlap)
        assert np.array_equal(dec.cpu().numpy().astype(bool), dec_ref), form
        assert np.array_equal(eye.cpu().numpy().astype(bool), OI.match_per_eye(dec_ref, W.n_shifts)), form


BATCH = [(0, W.d1), SHARD, (W.d1 - 1, 1), (0, W.d1)]


@pytest.mark.parametrize("form", ["i8", "rns", "p2"])
def test_mid_batched_items_bit_exact(mid, form):
    """Four items of the same query: two on the full range (one problem, 544 columns), a shard and
    the last code alone (split problems reading the A problem's query planes)."""
    _say(f"[gpu-mid] batched form {form}")
    items = [(mid["qct"], row0, rows) for row0, rows in BATCH]
    outs = H.hfe_ccmm_batched(mid["db"], items, FORMS[form])
    for k, ((row0, rows), r) in enumerate(zip(BATCH, outs)):
        _assert_equal(_result(r, rows), _expected(mid["c"], row0, rows), f"{form} batch item {k}")


@pytest.mark.parametrize("form", ["i8", "rns", "p2"])
def test_mid_plan_graph_replays_bit_exact(mid, form):
    _say(f"[gpu-mid] plan with captured graph, form {form}")
    plan = H.hfe_plan_create(mid["db"], len(BATCH), len(BATCH) * W.d3, W.level, FORMS[form])
    items = [(mid["qct"], row0, rows) for row0, rows in BATCH]
    for rep in range(3):
        H.hfe_plan_run(plan, items, use_graph=True)
        torch.cuda.synchronize()
        for k, (row0, rows) in enumerate(BATCH):
            got = _result(H.hfe_plan_result(plan, k), rows)
            _assert_equal(got, _expected(mid["c"], row0, rows), f"{form} replay {rep} item {k}")
        # eager work between replays
        H.hfe_ccmm(mid["db"], mid["qct"], *SHARD, FORMS[form])
        torch.cuda.synchronize()
