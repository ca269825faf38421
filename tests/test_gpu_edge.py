"""Edge shapes of the contraction at the limits of its exact integer arithmetic.

* K = d2 + N_Q beyond one exact int32 chunk of the digit form (511 K-blocks of 64 entries): the
  contraction runs in chunks whose partial results are added mod q, a path no other shape here
  reaches (K = 5,120 at the tiny shape, 20,992 at the share shape).
* K just below 2^17, the largest the RNS form accepts (int32 sums of 128 x 128 products), where it
  needs 12 small moduli instead of 11.

At both sizes the three forms must give the same residues (every digit tile configuration
included), and decryption must give exactly the plaintext products M_DB M_Q (computed with numpy
integers), with a ragged query count (d3 = 5) and database rows (d1 = 70).
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
