"""The allocation-free CCMM entry point (hfe_ccmm_noalloc) against hfe_ccmm.

hfe_ccmm_noalloc runs the same lift, contraction and rescale as hfe_ccmm with the call's buffers
carved from the library's static device array; its results must be the same residues, bit for bit,
in every form.  Two calls in a row: the mid workload (956 output rows, 272 query columns, three
query primes plus p), then a smaller one (a row shard and a 40-column, level-2 query), so the
second call reuses the array with the first call's contents still in it.  The first call is also
compared with the oracle.  A call whose buffers exceed the array is refused with HFE_ENOMEM and
writes nothing.
"""
import sys

import numpy as np
import pytest

import hfe_synth as S

from oracle_cases import DB_SEED, KEY_SEED, Q_SEED, case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")

FORMS = {"plain": H.HFE_FORM_PLAIN_U64, "i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}
W = S.MID


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    dev = torch.device("cuda", 0)
    _say(f"[no-alloc] {W.name}: keygen, encrypt database and queries")
    P = H.hfe_default_params(W.log_n_db, W.log_n_q, W.n_q_primes, W.d2, W.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    inp = S.make_inputs(W)
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(s) for s in inp["shifts"]]
    m_db = H.hfe_encode(torch.from_numpy(inp["db_codes"]).to(dev), db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, sum(FORMS.values()))
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), q_masks, shifts)
    q_full = H.hfe_encrypt(keys, m_q, W.level, Q_SEED)
    q_small = H.hfe_encrypt(keys, m_q[:40].contiguous(), 2, Q_SEED + 1)
    H.hfe_noalloc_init()
    torch.cuda.synchronize()
    return dict(keys=keys, db=db, q_full=q_full, q_small=q_small, m_q=m_q, n_db=1 << W.log_n_db)


def _noalloc(env, q, row0, rows, form):
    level, d3, _, _ = H.hfe_shape(q)
    out = torch.full((level, d3, env["n_db"] + rows), -1, dtype=torch.int64, device="cuda")
    H.hfe_ccmm_noalloc(env["db"], q, row0, rows, form, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _single(env, q, row0, rows, form):
    level, d3, _, _ = H.hfe_shape(q)
    r = H.hfe_ccmm(env["db"], q, row0, rows, form)
    return H.hfe_export(r, 0).reshape(level, d3, -1).astype(np.int64)


@pytest.mark.parametrize("form", list(FORMS))
def test_noalloc_equals_single_call_twice_in_a_row(env, form):
    f = FORMS[form]
    _say(f"[no-alloc] form {form}: full range, 272 columns, level 3")
    got1 = _noalloc(env, env["q_full"], 0, W.d1, f)
    exp1 = _single(env, env["q_full"], 0, W.d1, f)
    assert got1.shape == exp1.shape
    bad = np.argwhere(got1 != exp1)
    assert bad.size == 0, f"first call: {len(bad)} residues differ, first {bad[:3].tolist()}"
    _say(f"[no-alloc] form {form}: codes [150, 581), 40 columns, level 2")
    got2 = _noalloc(env, env["q_small"], 150, 431, f)
    exp2 = _single(env, env["q_small"], 150, 431, f)
    bad = np.argwhere(got2 != exp2)
    assert bad.size == 0, f"second call: {len(bad)} residues differ, first {bad[:3].tolist()}"


def test_noalloc_first_call_equals_the_oracle(env):
    c = case(W.name)
    _say("[no-alloc] digit form against the oracle")
    got = _noalloc(env, env["q_full"], 0, W.d1, H.HFE_FORM_I8_MFMA)
    for i in range(W.level):
        assert np.array_equal(got[i], c.out[i]), f"prime {i}: residues differ from the oracle"


@pytest.mark.parametrize("form", ["i8", "rns"])
def test_noalloc_refuses_a_call_beyond_the_array(env, form):
    """4,096 query columns need more than the 256 MiB array in the int8 forms (about 66 KB per
    column for the digit form and 121 KB for the RNS form on this database): HFE_ENOMEM, and the
    output is left untouched."""
    dev = torch.device("cuda", 0)
    g = torch.Generator().manual_seed(7)
    codes = torch.randint(0, 2, (256, W.d2), generator=g, dtype=torch.uint8).to(dev)
    masks = torch.ones((256, W.d2), dtype=torch.uint8, device=dev)
    m_q = H.hfe_encode(codes, masks, list(range(-8, 8)))
    q = H.hfe_encrypt(env["keys"], m_q, 3, Q_SEED + 2)
    out = torch.full((3, 4096, env["n_db"] + W.d1), 7, dtype=torch.int64, device=dev)
    _say(f"[no-alloc] form {form}: 4,096 columns (beyond the array)")
    with pytest.raises(H.HfeError) as ei:
        H.hfe_ccmm_noalloc(env["db"], q, 0, W.d1, FORMS[form], out)
    assert ei.value.status == -4  # HFE_ENOMEM
    torch.cuda.synchronize()
    assert bool((out == 7).all())
