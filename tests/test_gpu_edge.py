"""Edge shapes of the contraction at the limits of its exact integer arithmetic.

* K = d2 + N_Q beyond one exact int32 chunk of the digit form (511 K-blocks of 64 entries): the
  contraction runs in chunks whose partial results are added mod q, a path no other shape here
  reaches (K = 5,120 at the tiny shape, 20,992 at the share shape).
* K just below 2^17, the largest the RNS form accepts (int32 sums of 128 x 128 products), where it
  needs 12 small moduli instead of 11.

* K = 2^16, the largest the n^2 form accepts (int32 sums of 2 K products of digits up to 125).

At every size the forms must give the same residues (every digit tile configuration included), and
decryption must give exactly the plaintext products M_DB M_Q (computed with numpy integers), with a
ragged query count (d3 = 5) and database rows (d1 = 70).  Then the degenerate inputs: fully masked
codes, and empty row ranges and batches.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

FORMS = (H.HFE_FORM_PLAIN_U64, H.HFE_FORM_I8_MFMA, H.HFE_FORM_RNS_I8, H.HFE_FORM_P2_I8)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("d2", [32768, 65024, 130048],
                         ids=["k33280_two_digit_chunks", "k65536_n2_limit", "k130560_near_rns_limit"])
def test_long_k_all_forms_agree_and_decrypt_exactly(d2):
    log_n_db, log_n_q, d1, d3, level = 7, 9, 70, 5, 2
    K = d2 + (1 << log_n_q)
    assert K > 511 * 64 and K < 1 << 17
    forms = FORMS if K <= 1 << 16 else FORMS[:3]  # the n^2 form needs K <= 2^16
    _say(f"[gpu-edge] K = {K}: keygen, encrypt")
    dev = torch.device("cuda", 0)
    P = H.hfe_default_params(log_n_db, log_n_q, level, d2, d1)
    keys = H.hfe_keygen(P, 31)
    rng = np.random.default_rng(d2)
    m_db = rng.integers(-1, 2, (d1, d2)).astype(np.int8)
    m_q = rng.integers(-1, 2, (d3, d2)).astype(np.int8)
    if K > 1 << 16:
        with pytest.raises(H.HfeError):
            H.hfe_encrypt_db(keys, torch.from_numpy(m_db).to(dev), 32, H.HFE_FORM_P2_I8)
    db = H.hfe_encrypt_db(keys, torch.from_numpy(m_db).to(dev), 32, sum(forms))
    q = H.hfe_encrypt(keys, torch.from_numpy(m_q).to(dev), level, 33)
    exact = (m_q.astype(np.int64) @ m_db.astype(np.int64).T)  # d3 x d1
    ref = None
    for form in forms:
        _say(f"[gpu-edge] K = {K}: ccmm form {form}")
        r = H.hfe_ccmm(db, q, 0, d1, form)
        out = H.hfe_export(r, 0)
        ref = out if ref is None else ref
        assert np.array_equal(out, ref), f"form {form} differs from the plain form"
        _, ip = H.hfe_decrypt(keys, r, v=False)
        torch.cuda.synchronize()
        assert np.array_equal(ip.cpu().numpy(), exact), f"form {form}: decrypted products differ"
    for v in range(H.hfe_i8_variants()):
        _say(f"[gpu-edge] K = {K}: digit tile {H.hfe_i8_variant_name(v)}")
        H.hfe_set_i8_variant(v)
        try:
            out = H.hfe_export(H.hfe_ccmm(db, q, 0, d1, H.HFE_FORM_I8_MFMA), 0)
        finally:
            H.hfe_set_i8_variant(-1)
        assert np.array_equal(out, ref), f"tile {H.hfe_i8_variant_name(v)} differs"


def test_fully_masked_codes_decide_no_match_in_every_form():
    """Degenerate inputs of the method: query eyes and database codes whose masks are all zero
    (no usable bit), beside ordinary ones.  A masked pair has IP = 0 and overlap 0, so its score is
    undefined and the decision must be 'no match'; every other pair must still equal the popcount
    truth.  All four forms, full path (encode, encrypt, contraction, decrypt, match)."""
    from oracle import iris as OI
    log_n_db, log_n_q, d1, d2, level = 9, 10, 40, 512, 2
    n_eyes, shifts = 3, [0, 1, -2]
    rng = np.random.default_rng(77)
    db_codes = rng.integers(0, 2, (d1, d2)).astype(np.uint8)
    db_masks = (rng.random((d1, d2)) < 0.9).astype(np.uint8)
    q_codes = rng.integers(0, 2, (n_eyes, d2)).astype(np.uint8)
    q_masks = (rng.random((n_eyes, d2)) < 0.9).astype(np.uint8)
    db_masks[[0, 17, d1 - 1]] = 0                    # fully masked database codes
    q_masks[1] = 0                                   # a fully masked query eye
    db_codes[5] = q_codes[0]                         # and one exact match
    db_masks[5] = q_masks[0]
    qc, qm = OI.shifted_queries(q_codes, q_masks, np.array(shifts))
    ip_true, ov = OI.truth(qc, qm, db_codes, db_masks)
    dec_true = OI.decide(ip_true, ov)
    assert not dec_true[:, [0, 17, d1 - 1]].any() and not dec_true[3:6].any() and dec_true[0, 5]
    dev = torch.device("cuda", 0)
    P = H.hfe_default_params(log_n_db, log_n_q, level, d2, d1)
    keys = H.hfe_keygen(P, 41)
    t = {k: torch.from_numpy(v).to(dev) for k, v in
         dict(dc=db_codes, dm=db_masks, qc=q_codes, qm=q_masks).items()}
    _say("[gpu-edge] masked codes: encode, encrypt")
    db = H.hfe_encrypt_db(keys, H.hfe_encode(t["dc"], t["dm"], [0]), 42, sum(FORMS))
    q = H.hfe_encrypt(keys, H.hfe_encode(t["qc"], t["qm"], shifts), level, 43)
    for form in FORMS:
        _say(f"[gpu-edge] masked codes: form {form}")
        r = H.hfe_ccmm(db, q, 0, d1, form)
        _, ip = H.hfe_decrypt(keys, r, v=False)
        dec, eye = H.hfe_match(ip, t["qm"], shifts, t["dm"])
        torch.cuda.synchronize()
        assert np.array_equal(ip.cpu().numpy(), ip_true), f"form {form}: IP"
        assert np.array_equal(dec.cpu().numpy().astype(bool), dec_true), f"form {form}: decisions"
        assert np.array_equal(eye.cpu().numpy().astype(bool), OI.match_per_eye(dec_true, len(shifts)))


def test_empty_inputs_are_rejected():
    """Empty row ranges and empty batches are shape errors, not launches."""
    log_n_db, log_n_q, d1, d2, level = 7, 9, 8, 256, 1
    dev = torch.device("cuda", 0)
    P = H.hfe_default_params(log_n_db, log_n_q, level, d2, d1)
    keys = H.hfe_keygen(P, 5)
    m = torch.ones((d1, d2), dtype=torch.int8, device=dev)
    db = H.hfe_encrypt_db(keys, m, 6, sum(FORMS))
    q = H.hfe_encrypt(keys, m[:2].contiguous(), level, 7)
    for form in FORMS:
        with pytest.raises(H.HfeError) as e:
            H.hfe_ccmm(db, q, 0, 0, form)                          # no database rows
        assert e.value.status == -2
        with pytest.raises(H.HfeError) as e:
            H.hfe_ccmm(db, q, d1, 1, form)                         # range past the end
        assert e.value.status == -2
    with pytest.raises(H.HfeError) as e:
        H.hfe_ccmm_batched(db, [], H.HFE_FORM_I8_MFMA)              # empty batch
    assert e.value.status == -1
    with pytest.raises(H.HfeError) as e:
        H.hfe_ccmm_batched(db, [(q, 0, 0)], H.HFE_FORM_P2_I8)       # empty item
    assert e.value.status == -2


@pytest.mark.parametrize("bad", [2, -2, 127, -128], ids=["2", "-2", "127", "-128"])
def test_non_ternary_inputs_are_rejected(bad):
    """An entry outside {-1, 0, 1} would break the bound |M m| <= d2 that the scale leaves room
    for; both encryption calls refuse it, in the vector body and in the ragged tail of the check."""
    log_n_db, log_n_q, d1, d2, level = 7, 9, 9, 250, 1          # d1 x d2 and 3 x d2 not multiples of 16
    dev = torch.device("cuda", 0)
    keys = H.hfe_keygen(H.hfe_default_params(log_n_db, log_n_q, level, d2, d1), 8)
    rng = np.random.default_rng(bad & 0xff)
    for pos in (0, 1234 % (d1 * d2), d1 * d2 - 1):             # head, vector body, ragged tail
        m = rng.integers(-1, 2, (d1, d2)).astype(np.int8)
        m.reshape(-1)[pos] = bad
        with pytest.raises(H.HfeError) as e:
            H.hfe_encrypt_db(keys, torch.from_numpy(m).to(dev), 9, H.HFE_FORM_I8_MFMA)
        assert e.value.status == -1 and "outside" in str(e.value)
        q = np.ascontiguousarray(m[:3])
        if pos < 3 * d2:
            with pytest.raises(H.HfeError) as e:
                H.hfe_encrypt(keys, torch.from_numpy(q).to(dev), level, 10)
            assert e.value.status == -1
    ok = rng.integers(-1, 2, (d1, d2)).astype(np.int8)
    H.hfe_encrypt_db(keys, torch.from_numpy(ok).to(dev), 9, H.HFE_FORM_I8_MFMA)   # ternary: accepted
    H.hfe_encrypt(keys, torch.from_numpy(np.ascontiguousarray(ok[:3])).to(dev), level, 10)
