"""Parity at one GPU's share of the paper's workload (N_DB = 2^14, N_Q = 2^13, 3 query primes
plus p, 14,336 database codes x 512 query columns of 12,800 bits), in the launch
configuration the benchmark times.

The oracle cannot materialise this size, so the checks are:
  * keys: every secret coefficient equals the oracle's;
  * database and query ciphertexts: sampled entries (A-part and B-part rows, every prime,
    first/last/ragged columns) and whole sampled query columns equal the oracle's
    single-entry evaluation of the same definitions; 4,096 more database entries of 32 whole
    rows (16 of them B rows) equal the oracle's values stored in golden/share_samples.json;
  * CCMM result: 6,144 result residues (32 rows, A and B, x 64 columns, 8 in every 64-column
    tile, x 3 primes) equal the oracle's stored values, in every form and every digit tile
    configuration, on the full row range and on a row shard; sampled A-part entries are also
    recomputed here from the oracle's rows and columns; all four forms agree on every residue;
  * the exact product before the rescale, in every form, satisfies C r = D (X r) mod each prime
    for two random vectors r (Freivalds), with D the database residues and X the lifted query
    (the query residues, and for p their centered CRT value mod p computed by the oracle); and
    RS_p of 20,000 sampled product entries, by the oracle's big-integer rescale, equals the result;
  * decryption: every one of the 7,340,032 inner products equals the brute-force popcount
    truth and lies within 0.25 of it; decisions and per-eye matches agree.
"""
import json
import os
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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "share_samples.json")
SHARD = (3000, 5000)


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        g = json.load(f)
    assert g["workload"] == W.name and g["seeds"] == {"keys": KEY_SEED, "db": DB_SEED, "query": Q_SEED}
    g["result"] = np.array(g["result"], dtype=np.int64)      # [prime][col][row]
    g["db"] = np.array(g["db"], dtype=np.int64)              # [slot][row][k]
    return g


def test_golden_database_entries(run, golden):
    Po = run["Po"]
    R = Po.n_db + W.d1
    got = np.empty_like(golden["db"])
    for z in range(got.shape[0]):
        for a, r in enumerate(golden["rows"]):
            for b, k in enumerate(golden["db_cols"]):
                got[z, a, b] = int(H.hfe_export(run["db"], 0, (z * Po.K + k) * R + r, 1)[0])
    bad = np.argwhere(got != golden["db"])
    assert bad.size == 0, f"{len(bad)} database entries differ, first {bad[:3].tolist()}"


def _check_golden(res, golden, rows_out, what):
    """res: [prime][col][row] result residues; rows_out: output row of each golden row (or -1)."""
    cols = np.array(golden["cols"])
    sel = [a for a, r in enumerate(rows_out) if r >= 0]
    got = res[:, cols][:, :, [rows_out[a] for a in sel]]
    exp = golden["result"][:, :, sel]
    bad = np.argwhere(got != exp)
    assert bad.size == 0, f"{what}: {len(bad)} of {exp.size} sampled residues differ, first {bad[:3].tolist()}"
    return exp.size


@pytest.mark.parametrize("form", ["plain", "i8", "rns", "p2"])
def test_golden_sampled_results(run, golden, form):
    forms = {"plain": H.HFE_FORM_PLAIN_U64, "i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8,
             "p2": H.HFE_FORM_P2_I8}
    Po = run["Po"]
    n = Po.n_db
    rows_full = list(golden["rows"])
    # the shard's output rows: A rows as they are, codes in [row0, row0 + rows) shifted
    row0, rows = SHARD
    rows_shard = [r if r < n else (n + r - n - row0 if row0 <= r - n < row0 + rows else -1) for r in rows_full]
    configs = [None]
    if form == "i8":
        configs = list(range(H.hfe_i8_variants()))
    checked = 0
    try:
        for v in configs:
            if v is not None:
                H.hfe_set_i8_variant(v)
            for (r0, nr), rows_out in (((0, W.d1), rows_full), (SHARD, rows_shard)):
                tag = f"{form}" + (f" tile {H.hfe_i8_variant_name(v)}" if v is not None else "") + f" rows {r0}+{nr}"
                _say(f"[gpu-scale] golden samples: {tag}")
                r = H.hfe_ccmm(run["db"], run["qct"], r0, nr, forms[form])
                res = H.hfe_export(r, 0).reshape(W.level, W.d3, n + nr).astype(np.int64)
                checked += _check_golden(res, golden, rows_out, tag)
    finally:
        H.hfe_set_i8_variant(-1)
    assert checked >= 4096


_lift_p = {}


def _lifted_query(run, XT, prime):
    if prime not in _lift_p:
        _lift_p[prime] = OC.lift_mod(run["Po"], {i: XT[i] for i in range(W.level)}, W.level, prime)
    return _lift_p[prime]


def _matmul_mod(A, B, prime, chunk=2048):
    """(A @ B) mod prime for residue matrices (entries in [0, 2^36)), exactly: both operands are
    split into 18-bit limbs and each limb product is summed by a float64 matrix product.  Every limb
    product is an integer below 2^36 and every partial sum an integer below K 2^36 < 2^53, so each
    addition is exact in float64 whatever the summation order; the limbs are recombined with Python
    integers."""
    A = np.asarray(A)
    B = np.asarray(B)
    K = A.shape[1]
    assert B.shape[0] == K and K * (1 << 36) < (1 << 53)
    assert A.min() >= 0 and B.min() >= 0 and A.max() < (1 << 36) and B.max() < (1 << 36)
    m = (1 << 18) - 1
    acc = [np.zeros((A.shape[0], B.shape[1])) for _ in range(3)]
    for k0 in range(0, K, chunk):
        a = A[:, k0:k0 + chunk]
        b = B[k0:k0 + chunk]
        a0, a1 = (a & m).astype(np.float64), (a >> 18).astype(np.float64)
        b0, b1 = (b & m).astype(np.float64), (b >> 18).astype(np.float64)
        acc[0] += a0 @ b0
        acc[1] += a0 @ b1 + a1 @ b0
        acc[2] += a1 @ b1
    p0, p1, p2 = (x.astype(np.int64).astype(object) for x in acc)
    return ((p0 + p1 * (1 << 18) + p2 * (1 << 36)) % prime).astype(np.int64)


def test_freivalds_product_before_rescale_every_form(run):
    """C r = D (X r) mod prime for every prime, every form, two random vectors r."""
    Po = run["Po"]
    R = Po.n_db + W.d1
    K = Po.K
    XT = H.hfe_export(run["qct"], 0).reshape(W.level, W.d3, K).astype(np.int64)
    forms = {"plain": H.HFE_FORM_PLAIN_U64, "i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8,
             "p2": H.HFE_FORM_P2_I8}
    Cs = {}
    for name, f in forms.items():
        _say(f"[gpu-scale] product before rescale, form {name}")
        Cs[name] = H.hfe_ccmm_product(run["db"], run["qct"], 0, W.d1, f).cpu().numpy()
    run["C_i8"] = Cs["i8"]
    rng = np.random.default_rng(99)
    ids = OC.prime_ids(Po, W.level)
    for z, (pid, prime) in enumerate(ids):
        _say(f"[gpu-scale] Freivalds, prime slot {z}")
        X = XT[z] if z < W.level else _lifted_query(run, XT, prime)           # d3 x K
        rv = rng.integers(0, prime, (W.d3, 2), dtype=np.int64)
        y = _matmul_mod(X.T, rv, prime)                                        # K x 2
        Dt = H.hfe_export(run["db"], 0, z * K * R, K * R).astype(np.int64).reshape(K, R)
        rhs = _matmul_mod(y.T, Dt, prime).T                                    # R x 2: (D y) = (y^T D^T)^T
        del Dt
        for name, C in Cs.items():
            lhs = _matmul_mod(C[z].T, rv, prime)                               # R x 2
            bad = np.argwhere(lhs != rhs)
            assert bad.size == 0, f"{name} prime slot {z}: C r != D X r at {len(bad)} rows, first {bad[:3].tolist()}"


def test_rescale_of_sampled_product_entries(run):
    """RS_p by the oracle's big-integer CRT and rounding, on 20,000 sampled entries of the digit
    form's product, equals the result residues."""
    Po = run["Po"]
    C = run.get("C_i8")
    if C is None:
        C = H.hfe_ccmm_product(run["db"], run["qct"], 0, W.d1, H.HFE_FORM_I8_MFMA).cpu().numpy()
    res = H.hfe_export(run["r_i8"], 0).reshape(W.level, W.d3, -1).astype(np.int64)
    ids = OC.prime_ids(Po, W.level)
    moduli = [m for _, m in ids]
    Q = Po.Q(W.level)
    rng = np.random.default_rng(5)
    cc = rng.integers(0, W.d3, 20000)
    rr = rng.integers(0, C.shape[2], 20000)
    for c, r in zip(cc.tolist(), rr.tolist()):
        y = OC.rescale_p(OC.crt([int(C[z, c, r]) for z in range(len(ids))], moduli), Po.p, Q)
        assert [y % qi for qi in moduli[:-1]] == [int(res[i, c, r]) for i in range(W.level)], (c, r)
