"""The continuous-batching server: every request's result is the same alone and in the mix.

Requests of uneven size (and level) are decrypted to exactly the plaintext inner products
M_DB M_Q that the oracle computes, whether each runs alone on an idle server or in a burst
where the worker packs several into each step; a request larger than one step is rejected; a
small memory budget makes requests queue over several steps rather than fail.
"""
import sys

import numpy as np
import pytest

import hfe_synth as S
from oracle import ring as OR

from oracle_cases import DB_SEED, KEY_SEED, case

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
    _say("[gpu-serving] tinymulti: keygen / encrypt database")
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    db = H.hfe_encrypt_db(keys, torch.from_numpy(c.m_db).to(dev), DB_SEED,
                          H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8)
    rng = np.random.default_rng(11)
    reqs = []
    for i, d3 in enumerate([1, 7, 16, 33, 2, 40, 16, 5, 24, 3, 12, 9]):
        mq = rng.integers(-1, 2, (d3, w.d2)).astype(np.int8)
        level = 1 if i % 4 == 3 else 2
        q = H.hfe_encrypt(keys, torch.from_numpy(mq).to(dev), level, 900 + i)
        exact = OR.imatmul(c.m_db.astype(np.int64), mq.astype(np.int64).T).T   # d3 x d1
        reqs.append((q, mq, exact))
    torch.cuda.synchronize()
    return dict(c=c, keys=keys, db=db, reqs=reqs, dev=dev)


def _run(srv, env, idx, burst):
    outs, tickets = {}, {}
    for i in idx:
        q, mq, _ = env["reqs"][i]
        outs[i] = torch.full((mq.shape[0], env["c"].w.d1), -7, dtype=torch.int32, device=env["dev"])
        tickets[i] = H.hfe_server_submit(srv, q, outs[i])
        if not burst:
            H.hfe_server_wait(srv, tickets[i], 60000)
    for i in idx:
        H.hfe_server_wait(srv, tickets[i], 60000)
        assert H.hfe_server_poll(srv, tickets[i]) == 2
    return {i: o.cpu().numpy() for i, o in outs.items()}


FORMS = {"i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}


@pytest.mark.parametrize("form", ["i8", "rns", "p2"])
def test_same_result_alone_and_in_the_mix(env, form):
    _say(f"[gpu-serving] server ({form}): requests alone, then in a burst")
    srv = H.hfe_server_create(env["db"], 2 << 30, 64, 8, 2, 2, FORMS[form])
    idx = list(range(len(env["reqs"])))
    alone = _run(srv, env, idx, burst=False)
    st_alone = H.hfe_server_stats(srv)
    H.hfe_server_reset_stats(srv)
    mix = _run(srv, env, idx, burst=True)
    st_mix = H.hfe_server_stats(srv)
    for i in idx:
        exact = env["reqs"][i][2]
        assert np.array_equal(alone[i], exact), f"request {i} alone"
        assert np.array_equal(mix[i], alone[i]), f"request {i} in the mix"
    assert st_alone["completed"] == len(idx) and st_alone["steps"] == len(idx)
    assert st_mix["completed"] == len(idx) and st_mix["steps"] < len(idx)      # batched steps
    assert st_mix["mean_cols_per_step"] > st_alone["mean_cols_per_step"]
    assert 0 < st_mix["p50_ms"] <= st_mix["p99_ms"]
    srv.free()


@pytest.mark.parametrize("form", ["rns", "p2"])
def test_encrypted_results_equal_single_calls_and_decrypt_exactly(env, form):
    """Requests that take their result encrypted (the server uses no secret for them), mixed in
    one burst with requests decrypted by the server: every encrypted result equals the single
    hfe_ccmm call's residues and decrypts (by the key holder) to the plaintext products."""
    _say(f"[gpu-serving] server ({form}): encrypted results in a mixed burst")
    srv = H.hfe_server_create(env["db"], 2 << 30, 64, 8, 2, 2, FORMS[form])
    d1 = env["c"].w.d1
    results, tickets, outs = {}, {}, {}
    for i, (q, mq, _) in enumerate(env["reqs"]):
        if i % 2 == 0:
            results[i] = H.hfe_result_create(env["db"], q)
            tickets[i] = H.hfe_server_submit_encrypted(srv, q, results[i])
        else:
            outs[i] = torch.full((mq.shape[0], d1), -7, dtype=torch.int32, device=env["dev"])
            tickets[i] = H.hfe_server_submit(srv, q, outs[i])
    for i in tickets:
        H.hfe_server_wait(srv, tickets[i], 60000)
    for i, (q, mq, exact) in enumerate(env["reqs"]):
        if i in results:
            single = H.hfe_export(H.hfe_ccmm(env["db"], q, 0, d1, FORMS[form]), 0)
            assert np.array_equal(H.hfe_export(results[i], 0), single), f"request {i}: residues"
            _, ip = H.hfe_decrypt(env["keys"], results[i], v=False)
            torch.cuda.synchronize()
            assert np.array_equal(ip.cpu().numpy(), exact), f"request {i}: decrypted products"
        else:
            assert np.array_equal(outs[i].cpu().numpy(), exact), f"request {i}: server-decrypted products"
    with pytest.raises(H.HfeError) as e:                             # a result shaped for another query
        H.hfe_server_submit_encrypted(srv, env["reqs"][1][0], H.hfe_result_create(env["db"], env["reqs"][0][0]))
    assert e.value.status == -2
    srv.free()


def test_small_budget_queues_and_oversized_request_is_rejected(env):
    c = env["c"]
    # a budget that fits about 48 columns per step over 2 slots: the burst runs in several steps
    per_col = (3 * 5 * c.P.K // 64 * 64 + 3 * (c.P.n_db + c.w.d1) * 8 * 2 + 2 * c.w.d1 * 8)
    srv = H.hfe_server_create(env["db"], 2 * (48 * per_col + 8 * 127 * 3 * 5 * 1024 * 2), 48, 8, 2, 2)
    idx = list(range(len(env["reqs"])))
    mix = _run(srv, env, idx, burst=True)
    for i in idx:
        assert np.array_equal(mix[i], env["reqs"][i][2])
    st = H.hfe_server_stats(srv)
    assert st["steps"] >= 4 and st["mean_cols_per_step"] <= 48
    big = torch.from_numpy(np.ones((60, c.w.d2), dtype=np.int8)).to(env["dev"])
    qbig = H.hfe_encrypt(env["keys"], big, 2, 77)
    out = torch.empty((60, c.w.d1), dtype=torch.int32, device=env["dev"])
    t = H.hfe_server_submit(srv, qbig, out)
    with pytest.raises(H.HfeError) as e:
        H.hfe_server_wait(srv, t, 60000)
    assert e.value.status == -6
    assert H.hfe_server_stats(srv)["rejected"] == 1
    srv.free()


def test_long_burst_keeps_server_state_bounded_and_overlaps_steps(env):
    """A burst of 1,500 one-column requests: every result equals the plaintext product, the server
    holds at most its retention window of finished request records afterwards (older tickets are
    unknown), both slots held steps at once, and steps of the two slots overlapped on the device."""
    _say("[gpu-serving] server (rns): long burst of one-column requests")
    srv = H.hfe_server_create(env["db"], 2 << 30, 64, 8, 2, 2, H.HFE_FORM_RNS_I8)
    q, mq, exact = env["reqs"][0]
    assert mq.shape[0] == 1
    n, d1 = 1500, env["c"].w.d1
    out = torch.full((n, d1), -7, dtype=torch.int32, device=env["dev"])
    tickets = [H.hfe_server_submit(srv, q, out[i:i + 1]) for i in range(n)]
    H.hfe_server_drain(srv, 120000)
    st = H.hfe_server_stats(srv)
    _say(f"[gpu-serving] long burst: steps {st['steps']} retained {st['retained']} "
         f"max busy slots {st['max_busy_slots']} overlapping step pairs {st['overlap_pairs']}")
    assert np.array_equal(out.cpu().numpy(), np.broadcast_to(exact, (n, d1)))
    assert st["completed"] == n and st["retained"] <= 1024
    with pytest.raises(H.HfeError) as e:                            # forgotten: beyond the window
        H.hfe_server_poll(srv, tickets[0])
    assert e.value.status == -1
    assert H.hfe_server_poll(srv, tickets[-1]) == 2                 # within the window
    assert st["max_busy_slots"] == 2
    assert st["overlap_pairs"] >= 1
    srv.free()
