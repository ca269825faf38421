"""Batched CCMM (one persistent grouped launch), the reusable plan with its captured hipGraph,
and the tile autotuner, for both int8 forms (digits, small-modulus RNS).

Every item of a batch is its own CCMM (own level, column count and database row range); items
with the same level and row range share one problem (columns side by side), which the batch
below exercises with groups of two and three items.  Each item's residues must equal the
oracle's (for the oracle-computed case) and the single-call result bit for bit, and its
decrypted inner products must equal the exact plaintext products M_DB M_Q computed by the
oracle.  Graph replays are checked after eager work in between, on every replay.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

import hfe_synth as S
from oracle import ring as OR

from oracle_cases import DB_SEED, KEY_SEED, Q_SEED, case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)
H = pytest.importorskip("paper_2601_17561_amd")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    c = case(S.TINY_MULTI.name)
    w = c.w
    dev = torch.device("cuda", 0)
    _say("[gpu-batched] tinymulti: keygen / encrypt database")
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    m_db = torch.from_numpy(c.m_db).to(dev)
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED,
                          H.HFE_FORM_PLAIN_U64 | H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8)
    rng = np.random.default_rng(7)
    # items: (m_q rows, level, row0, rows); the first is the oracle case itself
    specs = [(c.m_q, 2, 0, w.d1, Q_SEED), (rng.integers(-1, 2, (3, w.d2)), 1, 10, 100, 501),
             (rng.integers(-1, 2, (130, w.d2)), 2, 0, 256, 502), (rng.integers(-1, 2, (1, w.d2)), 1, 255, 1, 503),
             (rng.integers(-1, 2, (64, w.d2)), 2, 128, 128, 504), (rng.integers(-1, 2, (5, w.d2)), 1, 10, 100, 505),
             (rng.integers(-1, 2, (2, w.d2)), 2, 0, w.d1, 506)]
    items, mqs = [], []
    for mq, level, row0, rows, seed in specs:
        mq = np.ascontiguousarray(mq.astype(np.int8))
        q = H.hfe_encrypt(keys, torch.from_numpy(mq).to(dev), level, seed)
        items.append((q, row0, rows))
        mqs.append(mq)
    torch.cuda.synchronize()
    return dict(c=c, keys=keys, db=db, items=items, mqs=mqs)


def _residues(r):
    return H.hfe_export(r, 0)


def _plain_product(env, i):
    _, row0, rows = env["items"][i]
    return OR.imatmul(env["c"].m_db[row0:row0 + rows].astype(np.int64), env["mqs"][i].astype(np.int64).T).T


_singles = {}


def _check_results(env, results, tag):
    c = env["c"]
    if not _singles:
        for i, (q, row0, rows) in enumerate(env["items"]):
            _singles[i] = _residues(H.hfe_ccmm(env["db"], q, row0, rows, H.HFE_FORM_I8_MFMA))
    singles = [_singles[i] for i in range(len(results))]
    for i, r in enumerate(results):
        got = _residues(r)
        assert np.array_equal(got, singles[i]), f"{tag}: item {i} differs from the single call"
        _, ip = H.hfe_decrypt(env["keys"], r)
        assert np.array_equal(ip.cpu().numpy(), _plain_product(env, i)), f"{tag}: item {i} decrypts wrong"
    # item 0 is the oracle case: compare with the oracle residues directly
    out0 = _residues(results[0]).reshape(c.w.level, c.m_q.shape[0], -1).astype(np.int64)
    for lv in range(c.w.level):
        assert np.array_equal(out0[lv], c.out[lv]), f"{tag}: oracle mismatch at prime {lv}"


@pytest.mark.parametrize("variant", [-1, 1])
def test_batched_i8_equals_single_calls_and_oracle(env, variant):
    _say(f"[gpu-batched] hfe_ccmm_batched i8 variant={variant}")
    H.hfe_set_i8_variant(variant)
    try:
        res = H.hfe_ccmm_batched(env["db"], env["items"], H.HFE_FORM_I8_MFMA)
        torch.cuda.synchronize()
        _check_results(env, res, f"batched variant {variant}")
    finally:
        H.hfe_set_i8_variant(-1)


def test_batched_rns_equals_single_calls_and_oracle(env):
    _say("[gpu-batched] hfe_ccmm_batched rns")
    res = H.hfe_ccmm_batched(env["db"], env["items"], H.HFE_FORM_RNS_I8)
    torch.cuda.synchronize()
    _check_results(env, res, "batched rns")


def test_single_rns_calls_equal_digit_form_on_every_item(env):
    # the items include d3 x R_out not divisible by 4 (1 column x 129 rows), where the CRT takes
    # its entry-by-entry path, and divisible ones, where it reads 4-byte residue words
    _say("[gpu-batched] single hfe_ccmm calls, rns form, every item")
    res = [H.hfe_ccmm(env["db"], q, row0, rows, H.HFE_FORM_RNS_I8) for q, row0, rows in env["items"]]
    torch.cuda.synchronize()
    n_db = env["c"].P.n_db
    assert any(mq.shape[0] * (n_db + it[2]) % 4 for mq, it in zip(env["mqs"], env["items"]))
    _check_results(env, res, "single rns")


def test_batched_n2_equals_single_calls_and_oracle(env):
    _say("[gpu-batched] hfe_ccmm_batched n^2")
    res = H.hfe_ccmm_batched(env["db"], env["items"], H.HFE_FORM_P2_I8)
    torch.cuda.synchronize()
    _check_results(env, res, "batched n^2")


def test_single_n2_calls_equal_digit_form_on_every_item(env):
    # the items include an odd d3 x R_out (1 column x 129 rows), where the n^2 CRT reads its 2-byte
    # residues one by one, and even ones, where it reads 4-byte words
    _say("[gpu-batched] single hfe_ccmm calls, n^2 form, every item")
    res = [H.hfe_ccmm(env["db"], q, row0, rows, H.HFE_FORM_P2_I8) for q, row0, rows in env["items"]]
    torch.cuda.synchronize()
    n_db = env["c"].P.n_db
    assert any(mq.shape[0] * (n_db + it[2]) % 2 for mq, it in zip(env["mqs"], env["items"]))
    _check_results(env, res, "single n^2")


def test_batched_plain_equals_i8(env):
    _say("[gpu-batched] hfe_ccmm_batched plain")
    a = H.hfe_ccmm_batched(env["db"], env["items"], H.HFE_FORM_PLAIN_U64)
    b = H.hfe_ccmm_batched(env["db"], env["items"], H.HFE_FORM_I8_MFMA)
    for x, y in zip(a, b):
        assert np.array_equal(_residues(x), _residues(y))


PLAN_FORMS = {"i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}


@pytest.mark.parametrize("form", ["i8", "rns", "p2"])
def test_plan_graph_replays(env, form):
    items = env["items"]
    _say(f"[gpu-batched] plan ({form}): eager run, graph capture, replays with eager work between")
    plan = H.hfe_plan_create(env["db"], 8, 512, 2, PLAN_FORMS[form])
    H.hfe_plan_run(plan, items, use_graph=False)
    torch.cuda.synchronize()
    _check_results(env, [H.hfe_plan_result(plan, i) for i in range(len(items))], "plan eager")
    for rep in range(3):
        H.hfe_plan_run(plan, items, use_graph=True)
        torch.cuda.synchronize()
        _check_results(env, [H.hfe_plan_result(plan, i) for i in range(len(items))], f"graph replay {rep}")
        # eager work between replays (other launches on the same stream)
        H.hfe_ccmm(env["db"], items[1][0], 0, 50, H.HFE_FORM_I8_MFMA)
        torch.cuda.synchronize()
    # a different batch through the same captured graph
    sub = [items[3], items[1]]
    H.hfe_plan_run(plan, sub, use_graph=True)
    torch.cuda.synchronize()
    for j, (q, row0, rows) in enumerate(sub):
        single = _residues(H.hfe_ccmm(env["db"], q, row0, rows, H.HFE_FORM_I8_MFMA))
        assert np.array_equal(_residues(H.hfe_plan_result(plan, j)), single)
    with pytest.raises(H.HfeError):
        H.hfe_plan_result(plan, 2)                                   # only 2 items in the last run
    big = [(items[2][0], 0, 256)] * 5                                # 650 columns > capacity 512
    assert len(items) <= 8
    with pytest.raises(H.HfeError) as e:
        H.hfe_plan_run(plan, big)
    assert e.value.status == -2


@pytest.mark.parametrize("form", ["i8", "rns", "p2"])
def test_plan_sized_for_the_batch(env, form):
    """hfe_plan_create_for sizes the workspace to exactly this batch: its graph replays equal the
    single calls and the oracle; a batch that needs more of any workspace is refused."""
    items = env["items"]
    _say(f"[gpu-batched] plan sized for the batch ({form}): graph capture and replays")
    plan = H.hfe_plan_create_for(env["db"], items, PLAN_FORMS[form])
    for rep in range(2):
        H.hfe_plan_run(plan, items, use_graph=True)
        torch.cuda.synchronize()
        _check_results(env, [H.hfe_plan_result(plan, i) for i in range(len(items))], f"sized plan replay {rep}")
    # fewer items that fit: the first two
    H.hfe_plan_run(plan, items[:2], use_graph=True)
    torch.cuda.synchronize()
    _check_results(env, [H.hfe_plan_result(plan, i) for i in range(2)], "sized plan, subset")
    # the 130-column item twice needs more columns than the whole batch holds
    with pytest.raises(H.HfeError) as e:
        H.hfe_plan_run(plan, [items[2]] * 7)
    assert e.value.status == -2


def test_autotune_records_and_roundtrips(env):
    q, row0, rows = env["items"][2]
    _say("[gpu-batched] autotune")
    best = H.hfe_autotune(env["db"], q, row0, rows, reps=1)
    assert 0 <= best < H.hfe_i8_variants()
    r = H.hfe_ccmm(env["db"], q, row0, rows, H.HFE_FORM_I8_MFMA)
    H.hfe_set_i8_variant(0)
    r0 = H.hfe_ccmm(env["db"], q, row0, rows, H.HFE_FORM_I8_MFMA)
    H.hfe_set_i8_variant(-1)
    assert np.array_equal(_residues(r), _residues(r0))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        H.hfe_autotune_save(path)
        text = open(path).read()
        assert H.hfe_i8_variant_name(best) in text
        H.hfe_autotune_load(path)
        with open(path, "w") as f:
            f.write("2 256 no_such_tile\n")
        with pytest.raises(H.HfeError):
            H.hfe_autotune_load(path)
