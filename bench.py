#!/usr/bin/env python3
"""Encrypted 1:N iris matching on one MI355X: code comparisons per second.

One step is one pass of the hot path over a batch of 32 query eyes x 16 cyclic shifts
(512 query columns) against the resident encrypted database of 14,336 codes of 12,800 bits
(N_DB = 2^14, N_Q = 2^13, three query primes plus the special prime):

    masked ternary encoding of the shifted query templates -> query encryption ->
    CCMM (centered lift + digit split, int8-MFMA contraction, rescale) -> decryption and
    decoding -> threshold decision per pair and match per eye.

The database is encrypted once before timing and stays in HBM.  Inputs (template bits) are
resident in HBM before the timed region.  The metric counts query columns x database codes
(every shift is one comparison).  The same step with the plain uint64 contraction is timed
for comparison, and the contraction kernel is timed with HIP events on its stream inside
every timed step for the roofline figure.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import hfe_synth as S  # noqa: E402

PEAK_I8_TOPS = 5000.0        # MI355X dense int8 MFMA, TOP/s
# Bytes beyond L2 per launch of the contraction on the share workload (d3 = 512), from rocprofv3
# FETCH_SIZE + WRITE_SIZE scaled by a 1 GiB copy (profiles/pmc_k_gemm_i8_dma_q128_r128_share_q512.md,
# profiles/pmc_k_gemm_i8_dma2_w2_share_q512.md); reported only for the kernels they were taken on.
MEASURED_TRAFFIC_GB = {"dma_q128_w2": 28.3, "dma_r128_w2": 30.4, "dma2_w2": 90.1,
                       # the 256-column RNS and n^2 contractions (profiles/pmc_k_gemm_rns_share_q512.md,
                       # profiles/pmc_k_gemm_p2_share_q512.md), fetch + write
                       "rns256": 36.6, "p2_256": 46.1}
KEY_SEED, DB_SEED, Q_SEED = 11, 22, 33


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_work(w: S.Workload):
    n_db, n_q = 1 << w.log_n_db, 1 << w.log_n_q
    R_out = n_db + w.d1
    K = w.d2 + n_q
    W = R_out * K * w.d3 * (w.level + 1)          # residue multiply-adds per CCMM
    return dict(R_out=R_out, K=K, residue_macs=W, i8_ops=2 * 25 * W)


def rns_moduli(w: S.Workload, qmax: int) -> int:
    """Small moduli the RNS form uses for this shape (the library's rule): the shortest prefix
    of its coprime list whose product is at least 4 K ((q - 1) / 2)^2 for the largest prime q."""
    import math
    mods = (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191)
    K = w.d2 + (1 << w.log_n_q)
    bound = 4 * K * ((qmax - 1) // 2) ** 2
    for n in range(1, len(mods) + 1):
        if math.prod(mods[:n]) >= bound:
            return n
    raise ValueError("contraction too long for the small moduli")


def p2_bases(w: S.Workload, qmax: int) -> int:
    """Bases n of the n^2 form for this shape (the library's rule): the shortest prefix of its
    prime list whose squares' product is at least 4 K ((q - 1) / 2)^2 for the largest prime q."""
    import math
    bases = (251, 241, 239, 233, 229, 227, 223, 211)
    K = w.d2 + (1 << w.log_n_q)
    bound = 4 * K * ((qmax - 1) // 2) ** 2
    for n in range(1, len(bases) + 1):
        if math.prod(b * b for b in bases[:n]) >= bound:
            return n
    raise ValueError("contraction too long for the n^2 bases")


def cpu_baseline(w: S.Workload, inp, rows_sample: int, cols_sample: int):
    """The oracle's CCMM (lift, exact contraction, CRT rescale) on a slice of the workload."""
    import torch
    from oracle import ckks as OC
    from oracle import iris as OI
    from oracle import params as OP
    from oracle import prng

    P = OP.make_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = OC.keygen(P, KEY_SEED)
    qc, qm = OI.shifted_queries(inp["q_codes"][:1], inp["q_masks"][:1], inp["shifts"][:cols_sample])
    mq = OI.ternary(qc, qm)
    XT = OC.encrypt_query(keys, mq, w.level, Q_SEED)
    # database rows of the sample: the first rows of D (A-part), drawn from the database stream
    log_rows = int(np.log2(rows_sample))
    Ps = OP.Params(log_n_db=log_rows, log_n_q=P.log_n_q, q=P.q, p=P.p, d2=P.d2, max_db_rows=P.max_db_rows)
    D = {pid: prng.uniform_matrix(DB_SEED, prng.DBA, pid, rows_sample, P.K, prime)
         for pid, prime in OC.prime_ids(P, len(P.q))}
    t0 = time.perf_counter()
    OC.ccmm(Ps, D, XT, w.level, 0, 0)
    dt = time.perf_counter() - t0
    work = algorithmic_work(w)
    # the full step needs R_out x d3 output residues per prime for d1 x d3 comparisons
    cmp_per_s = w.d1 * rows_sample * cols_sample / (dt * work["R_out"])
    return dict(value=cmp_per_s, unit="comparisons/s", cores=1, kind="oracle",
                sample=(f"oracle CCMM (centered CRT lift, exact int64-limb contraction, CRT rescale) of "
                        f"{rows_sample} database rows x {cols_sample} query columns x full K={P.K} x "
                        f"{w.level + 1} primes in {dt:.1f} s, scaled by rows {rows_sample}/{work['R_out']}; "
                        f"encryption and decryption not included; numpy int64 products, 1 thread "
                        f"(torch threads available: {torch.get_num_threads()})"),
                seconds=dt)


def encrypt_database(H, torch, w, forms):
    inp_db = S.db_templates(w.seed, w.d1, w.d2)
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    dev = torch.device("cuda", 0)
    m_db = H.hfe_encode(torch.from_numpy(inp_db[0]).to(dev), torch.from_numpy(inp_db[1]).to(dev), [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, forms)
    torch.cuda.synchronize()
    return keys, db


def encrypt_eyes(H, torch, keys, w, stream_id, eyes, level, shifts):
    dev = torch.device("cuda", 0)
    codes, masks = S.random_eyes(w.seed, stream_id, eyes, w.d2)
    m_q = H.hfe_encode(torch.from_numpy(codes).to(dev), torch.from_numpy(masks).to(dev), shifts)
    return H.hfe_encrypt(keys, m_q, level, Q_SEED + stream_id)


def run_batched(args, H, torch):
    """Uneven batch: items of 1-64 eyes x 16 shifts at levels 1-5 (2-6 primes with p) against
    database shards of 2,048-14,336 codes, as one batched call (grouped persistent launches; the
    workspace sized to the batch, which a plan would size for its worst case), against the same
    items as one hfe_ccmm call each, for the three int8 forms."""
    w = S.PAPER_SHARE_L5
    n_db, K = 1 << w.log_n_db, w.d2 + (1 << w.log_n_q)
    mix = S.batched_mix(w.seed, args.batch_items, w.d1, 64, w.n_q_primes, 2048)
    shifts = [int(x) for x in S.default_shifts(16)]
    log(f"batched: encrypting the {w.d1}-code database with {w.n_q_primes} query primes + p (int8 forms)")
    keys, db = encrypt_database(H, torch, w, H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8)
    items = []
    for i, it in enumerate(mix):
        items.append((encrypt_eyes(H, torch, keys, w, i, it.eyes, it.level, shifts), it.row0, it.rows))
    torch.cuda.synchronize()
    cols = sum(it.eyes * 16 for it in mix)
    macs = sum((n_db + it.rows) * K * it.eyes * 16 * (it.level + 1) for it in mix)
    comparisons = sum(it.rows * it.eyes * 16 for it in mix)
    log(f"batched: {len(mix)} items, {cols} query columns; autotuning the digit tile")
    # the plan looks the autotuner's table up by its largest level and mean column count
    tq = encrypt_eyes(H, torch, keys, w, 999, 32, w.n_q_primes, shifts)
    tuned = H.hfe_autotune(db, tq, 0, w.d1, reps=1)
    tq.free()
    qs, p_special = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1).primes()
    n_mod = rns_moduli(w, max(list(qs) + [p_special]))
    n_b = p2_bases(w, max(list(qs) + [p_special]))
    tiles = {"rns": f"rns 256 or 128 columns per problem, {n_mod} moduli",
             "p2": f"n^2 256 or 128 columns per problem, {n_b} bases"}
    for name, form, per_mac in (("i8", H.HFE_FORM_I8_MFMA, 50), ("rns", H.HFE_FORM_RNS_I8, 2 * n_mod),
                                ("p2", H.HFE_FORM_P2_I8, 2 * 3 * n_b)):
        torch.cuda.empty_cache()                            # the previous form's workspace
        res = H.hfe_ccmm_batched(db, items, form)           # warm-up (workspace into torch's cache)
        same = all(np.array_equal(H.hfe_export(res[i], 0, 0, 1 << 16),
                                  H.hfe_export(H.hfe_ccmm(db, q, r0, nr, form), 0, 0, 1 << 16))
                   for i, (q, r0, nr) in list(enumerate(items))[:4])
        del res
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for r in H.hfe_ccmm_batched(db, items, form):
                r.free()
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        t0 = time.perf_counter()
        for q, r0, nr in items:
            H.hfe_ccmm(db, q, r0, nr, form).free()
        torch.cuda.synchronize()
        seq_ms = (time.perf_counter() - t0) * 1e3
        tops = per_mac * macs / (plan_ms * 1e-3) / 1e12
        line = {"metric": "batched encrypted CCMM, comparisons/s (grouped persistent launches)",
                "value": comparisons / (plan_ms * 1e-3), "unit": "comparisons/s", "n_gpus": 1, "steps": args.steps,
                "higher_is_better": True, "form": name, "ms_per_batch": plan_ms, "int8_tops": tops,
                "frac_of_peak": tops / PEAK_I8_TOPS, "sequential_ms": seq_ms,
                "speedup_vs_sequential": seq_ms / plan_ms, "same_residues_as_single_calls": bool(same),
                "tile": H.hfe_i8_variant_name(tuned) if name == "i8" else tiles[name],
                "dtype": "i8", "data": "synthetic",
                "config": {"workload": "batched_" + w.name, "items": len(mix), "eyes": "1-64", "shifts": 16,
                           "levels": "1-5 query primes + p", "rows": "2048-14336", "columns": cols}}
        print(json.dumps(line), flush=True)


def run_serving(args, H, torch):
    """Poisson arrivals of 1-32 eyes x 16 shifts against the resident share database, through
    the continuous-batching server; throughput and arrival-to-result latency percentiles.

    Queries are encrypted before the timed window (clients encrypt on their side): one ciphertext
    per eye count 1..32 serves every request of that size, so a 10 s window at 200 req/s needs
    4.3 GB of query ciphertexts rather than one per request."""
    w = S.PAPER_SHARE
    shifts = [int(x) for x in S.default_shifts(16)]
    log(f"serving: encrypting the {w.d1}-code database (int8 form)")
    form = {"rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}.get(args.serve_form, H.HFE_FORM_I8_MFMA)
    keys, db = encrypt_database(H, torch, w, form)
    dev = torch.device("cuda", 0)
    pool = {e: encrypt_eyes(H, torch, keys, w, 1000 + e, e, w.level, shifts) for e in range(1, 33)}
    torch.cuda.synchronize()
    lines = []
    for rate in args.rates:
        n = max(8, int(rate * args.serve_seconds))
        t_arr, eyes = S.poisson_arrivals(w.seed + int(rate), n, rate, 32)
        encrypted = args.serve_results == "encrypted"
        if encrypted:
            # result handles are preallocated by the clients (level x columns x (N_DB + d1)
            # residues each): keep the first requests whose results fit 120 GiB
            per_req = [w.level * int(e) * 16 * ((1 << w.log_n_db) + w.d1) * 8 for e in eyes]
            n = max(8, min(n, int(np.searchsorted(np.cumsum(per_req), 120 << 30))))
            t_arr, eyes = t_arr[:n], eyes[:n]
        log(f"serving: {n} requests at {rate} req/s over {t_arr[-1]:.1f} s ({args.serve_results} results)")
        if encrypted:
            outs = [H.hfe_result_create(db, pool[int(e)]) for e in eyes]
        else:
            outs = [torch.empty((int(e) * 16, w.d1), dtype=torch.int32, device=dev) for e in eyes]
        srv = H.hfe_server_create(db, args.serve_budget_gib << 30, args.serve_cols, 64, 2, w.level, form)
        tickets = []
        t0 = time.perf_counter()
        for i in range(n):
            wait = t0 + t_arr[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            if encrypted:
                tickets.append(H.hfe_server_submit_encrypted(srv, pool[int(eyes[i])], outs[i]))
            else:
                tickets.append(H.hfe_server_submit(srv, pool[int(eyes[i])], outs[i]))
        log(f"serving: all {n} submitted after {time.perf_counter() - t0:.1f} s")
        H.hfe_server_drain(srv, 600000)
        dt = time.perf_counter() - t0
        st = H.hfe_server_stats(srv)
        srv.free()
        cmp = int(eyes.sum()) * 16 * w.d1
        line = {"metric": "encrypted 1:N serving, comparisons/s with continuous batching",
                "value": cmp / dt, "unit": "comparisons/s", "n_gpus": 1, "higher_is_better": True,
                "offered_req_per_s": rate, "requests": n, "served_req_per_s": n / dt, "seconds": dt,
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "service_p50_ms": st["service_p50_ms"],
                "service_p99_ms": st["service_p99_ms"], "steps": st["steps"],
                "mean_cols_per_step": st["mean_cols_per_step"], "max_queue": st["max_queue"],
                "rejected": st["rejected"], "form": args.serve_form, "results": args.serve_results,
                "latency": ("arrival -> encrypted result ready" if encrypted else "arrival -> decrypted products"),
                "dtype": "i8", "data": "synthetic",
                "config": {"workload": "serving_" + w.name, "eyes": "1-32", "shifts": 16,
                           "arrivals": f"poisson {rate}/s", "window_s": args.serve_seconds,
                           "max_cols_per_step": args.serve_cols, "slots": 2,
                           "mem_budget_gib": args.serve_budget_gib}}
        print(json.dumps(line), flush=True)
        lines.append(line)
        torch.cuda.synchronize()
        for o in outs:
            if encrypted:
                o.free()
        del outs
    return lines


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--workload", default=S.PAPER_SHARE.name, choices=sorted(S.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=8192)
    ap.add_argument("--cpu-cols", type=int, default=32)
    ap.add_argument("--sweep", action="store_true", help="time every int8 tile configuration and exit")
    ap.add_argument("--variant", type=int, default=-1, help="int8 tile configuration (-1: default)")
    ap.add_argument("--ccmm-only", type=int, default=0, help="run N int8 CCMMs after setup and exit (profiling)")
    ap.add_argument("--form", choices=("i8", "rns", "p2"), default="i8", help="with --ccmm-only: the int8 form to run")
    ap.add_argument("--mode", choices=("step", "batched", "serving"), default="step",
                    help="step: the hot-path step (default); batched: 64 uneven items as one plan; "
                         "serving: Poisson arrivals through the server")
    ap.add_argument("--batch-items", type=int, default=64)
    ap.add_argument("--rates", type=float, nargs="+", default=[200.0, 50.0, 25.0],
                    help="serving arrival rates, req/s")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="serving: seconds of arrivals per rate")
    ap.add_argument("--serve-cols", type=int, default=2048, help="serving: query columns per step")
    ap.add_argument("--serve-results", choices=("decrypted", "encrypted"), default="decrypted",
                    help="serving: products decrypted by the server, or encrypted results for the key holder")
    ap.add_argument("--serve-budget-gib", type=int, default=64, help="serving: workspace memory budget")
    ap.add_argument("--serve-form", choices=("i8", "rns", "p2"), default="rns", help="serving: int8 form of the server")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="with --ccmm-only: also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU layout "
                                   "(database-row shards with a broadcast of the A-part result) is not built"}))
        sys.exit(2)

    import torch
    import paper_2601_17561_amd as H

    if args.mode == "batched":
        return run_batched(args, H, torch)
    if args.mode == "serving":
        return run_serving(args, H, torch)
    w = S.WORKLOADS[args.workload]
    work = algorithmic_work(w)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    log(f"workload {w.name}: d1={w.d1} d2={w.d2} d3={w.d3} N_DB=2^{w.log_n_db} N_Q=2^{w.log_n_q} "
        f"primes={w.level}+p")
    inp = S.make_inputs(w)
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    db_codes = torch.from_numpy(inp["db_codes"]).to(dev)
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_codes = torch.from_numpy(inp["q_codes"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(s) for s in inp["shifts"]]
    log("encrypting the database (plain, digit, RNS and n^2 forms)")
    t0 = time.perf_counter()
    m_db = H.hfe_encode(db_codes, db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED,
                          H.HFE_FORM_PLAIN_U64 | H.HFE_FORM_I8_MFMA | H.HFE_FORM_RNS_I8 | H.HFE_FORM_P2_I8)
    torch.cuda.synchronize()
    t_db = time.perf_counter() - t0
    del m_db
    log(f"database encrypted in {t_db:.2f} s")

    def step(form, profile_out=None, marks=None):
        # marks: 6 events recorded on the stream the library runs on (torch's current stream)
        # around encode, encrypt, CCMM, decrypt and match
        mark = (lambda i: marks[i].record()) if marks is not None else (lambda i: None)
        mark(0)
        m_q = H.hfe_encode(q_codes, q_masks, shifts)
        mark(1)
        qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
        mark(2)
        r = H.hfe_ccmm(db, qct, 0, w.d1, form)
        mark(3)
        _, ip = H.hfe_decrypt(keys, r, v=False)
        mark(4)
        _, eye = H.hfe_match(ip, q_masks, shifts, db_masks, want_decision=False)
        mark(5)
        if profile_out is not None:
            profile_out.append(r)
        else:
            r.free()
        qct.free()
        return ip, eye

    H.hfe_set_i8_variant(args.variant)
    tile = None
    if args.variant < 0 and not args.sweep and not args.ccmm_only:
        # the autotuner picks the int8 tile for this shape (setup, not timed)
        m_q = H.hfe_encode(q_codes, q_masks, shifts)
        qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
        tile = H.hfe_i8_variant_name(H.hfe_autotune(db, qct, 0, w.d1, reps=3))
        qct.free()
        log(f"autotuned int8 tile: {tile}")
    elif args.variant >= 0:
        tile = H.hfe_i8_variant_name(args.variant)
    if args.ccmm_only:
        m_q = H.hfe_encode(q_codes, q_masks, shifts)
        qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
        form = {"rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}.get(args.form, H.HFE_FORM_I8_MFMA)
        for _ in range(args.ccmm_only):
            H.hfe_ccmm(db, qct, 0, w.d1, form).free()
        torch.cuda.synchronize()
        log(f"ran {args.ccmm_only} int8 CCMMs")
        if args.copy_mib:
            src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev)
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            log(f"copied {args.copy_mib} MiB")
        return

    if args.sweep:
        m_q = H.hfe_encode(q_codes, q_masks, shifts)
        qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
        ref = None
        for v in range(H.hfe_i8_variants()):
            H.hfe_set_i8_variant(v)
            H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_I8_MFMA).free()
            H.hfe_profile(True)
            rs = [H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_I8_MFMA) for _ in range(3)]
            H.hfe_profile(False)
            ms = [H.hfe_profile_ms(r, 3)[1] for r in rs]
            out = H.hfe_export(rs[0], 0, 0, 1 << 20)
            ref = out if ref is None else ref
            ok = bool(np.array_equal(out, ref))
            print(json.dumps({"variant": H.hfe_i8_variant_name(v), "contraction_ms": min(ms),
                              "frac_of_peak": work["i8_ops"] / (min(ms) * 1e-3) / 1e12 / PEAK_I8_TOPS,
                              "same_residues": ok}), flush=True)
            for r in rs:
                r.free()
        return

    results = {}
    for name, form, steps, warm in (("i8", H.HFE_FORM_I8_MFMA, args.steps, args.warmup),
                                    ("rns", H.HFE_FORM_RNS_I8, args.steps, args.warmup),
                                    ("p2", H.HFE_FORM_P2_I8, args.steps, args.warmup),
                                    ("plain", H.HFE_FORM_PLAIN_U64, args.plain_steps, 1)):
        if steps <= 0:
            continue
        for _ in range(warm):
            step(form)
        torch.cuda.synchronize()
        H.hfe_profile(True)
        prof = []
        marks = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ip, eye = step(form, prof, marks[i])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        H.hfe_profile(False)
        stages = np.array([H.hfe_profile_ms(r, 3) for r in prof])
        phases = np.array([[m[k].elapsed_time(m[k + 1]) for k in range(5)] for m in marks])
        for r in prof:
            r.free()
        ms = dt * 1e3 / steps
        results[name] = dict(ms_per_step=ms, comparisons_per_s=w.d1 * w.d3 / (dt / steps),
                             lift_ms=float(stages[:, 0].mean()), contraction_ms=float(stages[:, 1].mean()),
                             contraction_median_ms=float(np.median(stages[:, 1])),
                             rescale_ms=float(stages[:, 2].mean()), ip=ip, eye=eye,
                             phases_ms={k: float(v) for k, v in zip(
                                 ("encode", "encrypt", "ccmm", "decrypt", "match"), phases.mean(axis=0))})
        log(f"{name}: {ms:.2f} ms/step, contraction {results[name]['contraction_ms']:.2f} ms "
            f"(lift {results[name]['lift_ms']:.2f}, rescale {results[name]['rescale_ms']:.2f}); phases "
            + " ".join(f"{k} {v:.3f}" for k, v in results[name]["phases_ms"].items()))

    plain = results.get("plain")
    same = bool(torch.equal(results["i8"]["ip"], plain["ip"])) if plain else None
    same_rns = bool(torch.equal(results["rns"]["ip"], results["i8"]["ip"]))
    rns = results["rns"]
    qs, p_special = P.primes()
    n_mod = rns_moduli(w, max(list(qs) + [p_special]))
    rns_ops = 2 * n_mod * work["residue_macs"]
    p2 = results["p2"]
    n_b = p2_bases(w, max(list(qs) + [p_special]))
    p2_ops = 2 * 3 * n_b * work["residue_macs"]
    same_p2 = bool(torch.equal(p2["ip"], results["i8"]["ip"]))
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        cpu = cpu_baseline(w, inp, args.cpu_rows, args.cpu_cols)
        cpu.pop("seconds")

    i8 = results["i8"]
    achieved = work["i8_ops"] / (i8["contraction_ms"] * 1e-3) / 1e12
    line = {
        "metric": "encrypted query x db code comparisons/sec on 1 MI355X, int8-MFMA vs plain",
        "value": i8["comparisons_per_s"],
        "unit": "comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": i8["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": w.name, "n_db": 1 << w.log_n_db, "n_q": 1 << w.log_n_q,
                   "query_primes": w.level, "special_primes": 1, "prime_bits": 36, "d1": w.d1, "d2": w.d2,
                   "eyes": w.eyes, "shifts": w.n_shifts, "d3": w.d3, "form": "i8_mfma",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_I8_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_I8_TOPS,
                     "traffic": (MEASURED_TRAFFIC_GB.get(tile) if w.name == S.PAPER_SHARE.name else None),
                     "traffic_unit": "GB per launch (HBM side of L2, rocprofv3 counters)",
                     "kernel": f"k_gemm_i8 ({tile})", "ops_per_launch": work["i8_ops"],
                     "kernel_ms": i8["contraction_ms"]},
        "plain": ({"ms_per_step": plain["ms_per_step"],
                   "comparisons_per_s": plain["comparisons_per_s"],
                   "contraction_ms": plain["contraction_ms"],
                   "residue_macs_per_s": work["residue_macs"] / (plain["contraction_ms"] * 1e-3)}
                  if plain else None),
        "rns": {"form": f"small-modulus RNS, {n_mod} moduli per prime", "ms_per_step": rns["ms_per_step"],
                "comparisons_per_s": rns["comparisons_per_s"], "contraction_ms": rns["contraction_ms"],
                "lift_ms": rns["lift_ms"], "crt_rescale_ms": rns["rescale_ms"],
                "int8_ops_per_launch": rns_ops,
                "traffic_gb": MEASURED_TRAFFIC_GB["rns256"] if w.name == S.PAPER_SHARE.name else None,
                "frac_of_peak": rns_ops / (rns["contraction_ms"] * 1e-3) / 1e12 / PEAK_I8_TOPS,
                "over_i8_step": i8["ms_per_step"] / rns["ms_per_step"], "equals_i8_ip": same_rns,
                "phases_ms": rns["phases_ms"]},
        "p2": {"form": f"n^2 split M + n M', {n_b} bases, 3 int8 products each, per prime",
               "ms_per_step": p2["ms_per_step"], "comparisons_per_s": p2["comparisons_per_s"],
               "contraction_ms": p2["contraction_ms"], "lift_ms": p2["lift_ms"], "crt_rescale_ms": p2["rescale_ms"],
               "int8_ops_per_launch": p2_ops,
               "traffic_gb": MEASURED_TRAFFIC_GB["p2_256"] if w.name == S.PAPER_SHARE.name else None,
               "frac_of_peak": p2_ops / (p2["contraction_ms"] * 1e-3) / 1e12 / PEAK_I8_TOPS,
               "over_i8_step": i8["ms_per_step"] / p2["ms_per_step"], "equals_i8_ip": same_p2,
               "phases_ms": p2["phases_ms"]},
        "i8_over_plain_step": plain["ms_per_step"] / i8["ms_per_step"] if plain else None,
        "stages_ms": {"lift_split": i8["lift_ms"], "contraction": i8["contraction_ms"],
                      "contraction_median": i8["contraction_median_ms"], "rescale": i8["rescale_ms"]},
        "phases_ms": i8["phases_ms"],
        "i8_equals_plain_ip": same,
        "db_encrypt_s": t_db,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
