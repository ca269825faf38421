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
# profiles/pmc_k_gemm_i8_dma2_w2_share_q512.md, profiles/pmc_k_gemm_i8_dmas_share_q512.md); reported only
# for the kernels they were taken on, and None for a tile whose kernel changed after its counters were taken.
MEASURED_TRAFFIC_GB = {"dma_q128_w2": 27.8, "dma_r128_w2": None, "dma2_w2": None,
                       "dmas_q128_w2": 27.3, "dmas_r128_w2": 27.5,
                       # the 256-column RNS and n^2 contractions (profiles/pmc_k_gemm_rns_share_q512.md,
                       # profiles/pmc_k_gemm_p2_share_q512.md), fetch + write
                       "rns256": 36.4, "p2_256": 43.9}
KEY_SEED, DB_SEED, Q_SEED, TX_SEED, FOLD_SEED = 11, 22, 33, 44, 55
# fp64 vector instructions per second of the chip (256 CUs x 64 lanes x 2.4 GHz; the 78.6 TFLOP/s peak
# counts a fused multiply-add as two) and the fp64 instructions of one exact modular product in the
# signed form the FormatSwitch transforms use (multiply, fused multiply-add, multiply by 1/q, rint,
# fused multiply-add, add): the ceiling of the modular products FormatSwitch is built from.
FP64_INSTR_PER_S = 256 * 64 * 2.4e9
FP64_PER_MODMUL = 6


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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_block(args):
    """One worker of the oracle contraction: its block of database rows (uniform residues per
    prime, not timed; the oracle's work does not depend on their values), then the oracle's CCMM
    of that block (timed), started together with the other workers at a barrier."""
    w, P, XT, row_lo, rows, barrier = args
    from oracle import ckks as OC
    from oracle import params as OP
    rng = np.random.default_rng(row_lo)
    D = {pid: rng.integers(0, prime, (rows, P.K), dtype=np.int64) for pid, prime in OC.prime_ids(P, w.level)}
    Ps = OP.Params(log_n_db=int(np.log2(rows)), log_n_q=P.log_n_q, q=P.q, p=P.p, d2=P.d2,
                   max_db_rows=P.max_db_rows)
    barrier.wait()
    t0 = time.perf_counter()
    OC.ccmm(Ps, D, XT, w.level, 0, 0)
    return time.perf_counter() - t0


def cpu_baseline(w: S.Workload, inp, workers: int, rows_per_worker: int, cols: int, enc_cols: int,
                 dec_rows: int):
    """The oracle timed on the host: query encryption of enc_cols columns, the CCMM (lift, exact
    contraction, CRT rescale) of workers x rows_per_worker database rows x cols query columns in a
    process pool (one row block per worker, started together), and decryption of cols columns x
    dec_rows codes; each part scaled linearly to the workload's columns and rows, summed per step.
    Runs before the GPU is touched, so the pool's fork copies no device state."""
    import multiprocessing as mp
    from oracle import ckks as OC
    from oracle import iris as OI
    from oracle import params as OP

    from oracle import prng

    P = OP.make_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = OC.keygen(P, KEY_SEED)
    qc, qm = OI.shifted_queries(inp["q_codes"][:2], inp["q_masks"][:2], inp["shifts"])
    mq = OI.ternary(qc, qm)
    SQ = OC.s_q_matrix(keys)  # the secret matrix: key set-up, built once (as the library's keygen tables)
    t0 = time.perf_counter()
    A = {i: prng.uniform_matrix(Q_SEED, prng.QA, i, P.n_q, enc_cols, P.q[i]) for i in range(w.level)}
    E = prng.gaussian_matrix(Q_SEED, prng.QE, 0, P.d2, enc_cols)
    OC.encrypt_query_with(P, SQ, mq[:enc_cols], w.level, A, E)
    t_enc = time.perf_counter() - t0
    XT = OC.encrypt_query(keys, mq[:cols], w.level, Q_SEED)
    t0 = time.perf_counter()
    OC.lift_query(P, XT, w.level)
    t_lift = time.perf_counter() - t0  # per query column; every worker repeats it for its block
    ctx = mp.get_context("fork")
    barrier = ctx.Manager().Barrier(workers)
    with ctx.Pool(workers) as pool:
        times = pool.map(_oracle_block, [(w, P, XT, i * rows_per_worker, rows_per_worker, barrier)
                                         for i in range(workers)])
    t_ccmm = max(times)
    t_rows = max(t_ccmm - t_lift, 0.0)  # the row-dependent part: contraction and CRT rescale
    # decryption of the sample: A_out for cols columns over the N_DB A rows, B_out for dec_rows codes
    rng = np.random.default_rng(5)
    out = {i: np.concatenate([rng.integers(0, P.q[i], (cols, P.n_db)), rng.integers(0, P.q[i], (cols, dec_rows))],
                             axis=1).astype(np.int64) for i in range(w.level)}
    t0 = time.perf_counter()
    OC.decrypt(keys, out, w.level, 0, dec_rows)
    t_dec = time.perf_counter() - t0
    work = algorithmic_work(w)
    step_s = (t_enc * w.d3 / enc_cols
              + t_lift * w.d3 / cols
              + t_rows * (work["R_out"] / (workers * rows_per_worker)) * (w.d3 / cols)
              + t_dec * (w.d1 / dec_rows) * (w.d3 / cols))
    return dict(value=w.d1 * w.d3 / step_s, unit="comparisons/s", cores=workers, kind="oracle",
                cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
                sample=(f"oracle step extrapolated from samples: query encryption of {enc_cols} columns in "
                        f"{t_enc:.1f} s (1 core, secret matrix prebuilt); CCMM centered CRT lift of {cols} "
                        f"columns in {t_lift:.1f} s (1 core); exact int64-limb contraction and CRT rescale of "
                        f"{workers} x {rows_per_worker} database rows x {cols} columns x full K={P.K} x "
                        f"{w.level + 1} primes in {t_rows:.1f} s ({workers} processes, one row block each, "
                        f"their lift time subtracted); decryption of {cols} columns x {dec_rows} codes in "
                        f"{t_dec:.1f} s (1 core); scaled linearly to {w.d3} columns, {work['R_out']} "
                        f"contraction rows and {w.d1} codes: {step_s:.0f} s per step"),
                parts_s={"encrypt": t_enc, "lift": t_lift, "contraction_rescale": t_rows, "decrypt": t_dec},
                step_s=step_s)


def _cpu_chain(args):
    """The chain oracle's CCMM (lift, exact products mod every n^2, CRT and RS_P) on rows x cols of the
    share shape (uniform residues: the oracle's work does not depend on their values), one core."""
    w, chain_q, rows, cols = args
    from oracle import chain as OCH
    rng = np.random.default_rng(9)
    C = OCH.make_chain_params(int(np.log2(rows)), w.log_n_q, chain_q, 3, w.d2, w.d1)
    D = {n: rng.integers(0, n * n, (rows, C.K), dtype=np.int64) for n in C.all_bases()}
    XT = {n: rng.integers(0, n * n, (cols, C.K), dtype=np.int64) for n in C.q_bases}
    t0 = time.perf_counter()
    OCH.lift_query(C, XT, chain_q)
    t_lift = time.perf_counter() - t0  # per query column; the CCMM below repeats it
    t0 = time.perf_counter()
    OCH.ccmm(C, D, XT, chain_q, 0, 0)
    return t_lift, max(time.perf_counter() - t0 - t_lift, 0.0), C.K


def _cpu_fs(args):
    """The FormatSwitch oracle on one query column of the share workload from ring degree 2^16, one
    core: keys, transmission encryption and the switch timed apart."""
    inp, = args
    from oracle import formatswitch as FS
    from oracle import iris as OI
    from oracle import params as OP
    fw = S.FS_SHARE
    P = OP.make_params(fw.log_n_db, fw.log_n_q, fw.n_q_primes, fw.d2, fw.d1)
    t0 = time.perf_counter()
    F = FS.fs_keygen(P, fw.level, S.FS_LOG_N_T[fw.name], KEY_SEED)
    t_keys = time.perf_counter() - t0
    qc, qm = OI.shifted_queries(inp["q_codes"][:1], inp["q_masks"][:1], inp["shifts"][:1])
    t0 = time.perf_counter()
    ct = FS.encrypt_transmit(F, OI.ternary(qc, qm), TX_SEED)
    t_tx = time.perf_counter() - t0
    t0 = time.perf_counter()
    FS.format_switch(F, ct, 1)
    return t_keys, t_tx, time.perf_counter() - t0


def _cpu_fold(args):
    """The fold oracle at the share workload's ring degree 2^14 on one group of `cts` score ciphertexts
    (one core): keys and encryption untimed, the fold timed."""
    cts, = args
    from oracle import fold as OF
    fw = S.FOLD_SHARE
    P = OF.fold_params(fw.log_n, fw.k)
    FK = OF.fold_keygen(P, KEY_SEED, OF.rot_amounts(fw.k, cts))
    ip, counts = S.fold_inputs(fw)
    enc = [OF.encrypt(FK, ip[c].astype(np.int64), FOLD_SEED, c) for c in range(cts)]
    t0 = time.perf_counter()
    OF.fold(FK, enc, counts[:cts].astype(np.int64), cts)
    return time.perf_counter() - t0


def cpu_baseline_chain_fs(w: S.Workload, inp, chain_q: int, rows: int = 128, cols: int = 4, fold_cts: int = 2):
    """The oracle beside three more measurements, in three processes side by side (one core each): the n^2
    chain's CCMM on a sample scaled to the step's rows and columns, FormatSwitch of one query column
    scaled to the workload's columns, and the fold of a group of `fold_cts` score ciphertexts scaled to the
    fold workload's ciphertexts.  Runs before the GPU is touched."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(3) as pool:
        rc = pool.apply_async(_cpu_chain, ((w, chain_q, rows, cols),))
        rf = pool.apply_async(_cpu_fs, ((inp,),))
        rd = pool.apply_async(_cpu_fold, ((fold_cts,),))
        t_lift, t_rows, K = rc.get()
        t_keys, t_tx, t_fs = rf.get()
        t_fold = rd.get()
    work = algorithmic_work(w)
    chain_step = t_lift * (w.d3 / cols) + t_rows * (work["R_out"] / rows) * (w.d3 / cols)
    chain = dict(value=w.d1 * w.d3 / chain_step, unit="comparisons/s", cores=1, kind="oracle",
                 sample=(f"the chain oracle's CCMM of {rows} database rows x {cols} columns x full K={K} over "
                         f"{chain_q} + 3 moduli n^2 (1 core): centered lift of the {cols} columns {t_lift:.1f} s, "
                         f"exact products, CRT and RS_P {t_rows:.1f} s; scaled to {work['R_out']} rows and "
                         f"{w.d3} columns: {chain_step:.0f} s per CCMM (encryption and decryption not included)"))
    fw = S.FS_SHARE
    fs = dict(value=1.0 / t_fs, unit="columns/s", cores=1, kind="oracle",
              sample=(f"the FormatSwitch oracle on one query column of the share workload (2^16 -> 2^13, level "
                      f"{fw.level}): keys {t_keys:.1f} s, transmission encryption {t_tx:.1f} s, the switch "
                      f"{t_fs:.1f} s (1 core); {t_fs * fw.d3:.0f} s for the {fw.d3} columns"))
    dw = S.FOLD_SHARE
    fold = dict(value=fold_cts / t_fold, unit="ciphertexts/s", cores=1, kind="oracle",
                sample=(f"the fold oracle at ring degree 2^{dw.log_n} on a group of {fold_cts} score ciphertexts "
                        f"(normalisation, f, {fold_cts - 1} rotation, the rescale; keys and encryption untimed): "
                        f"{t_fold:.1f} s (1 core); {t_fold / fold_cts * dw.count:.0f} s for the {dw.count} "
                        f"ciphertexts"))
    return chain, fs, fold


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


def run_batched(args, H, torch, forms=("i8", "rns", "p2"), steps=None, compare_sequential=True):
    """Uneven batch (configuration 4): items of 1-64 eyes x 16 shifts at levels 1-5 (2-6 primes
    with p) against database shards of 2,048-14,336 codes, run through a plan sized for the batch:
    one grouped lift launch, ONE persistent contraction launch over every item's tiles, the grouped
    reconstruction (small-modulus forms) and rescale, captured once into a hipGraph that every timed
    run replays.  Optionally the same items as one hfe_ccmm call each.  Returns one dict per form."""
    w = S.PAPER_SHARE_L5
    steps = steps or args.steps
    n_db, K = 1 << w.log_n_db, w.d2 + (1 << w.log_n_q)
    mix = S.batched_mix(w.seed, args.batch_items, w.d1, 64, w.n_q_primes, 2048)
    shifts = [int(x) for x in S.default_shifts(16)]
    codes = {"i8": H.HFE_FORM_I8_MFMA, "rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}
    log(f"batched: encrypting the {w.d1}-code database with {w.n_q_primes} query primes + p ({', '.join(forms)})")
    keys, db = encrypt_database(H, torch, w, sum(codes[f] for f in forms))
    items = []
    for i, it in enumerate(mix):
        items.append((encrypt_eyes(H, torch, keys, w, i, it.eyes, it.level, shifts), it.row0, it.rows))
    torch.cuda.synchronize()
    cols = sum(it.eyes * 16 for it in mix)
    macs = sum((n_db + it.rows) * K * it.eyes * 16 * (it.level + 1) for it in mix)
    comparisons = sum(it.rows * it.eyes * 16 for it in mix)
    tuned = None
    if "i8" in forms:
        log(f"batched: {len(mix)} items, {cols} query columns; autotuning the digit tile")
        # plans look the autotuner's table up by the batch's largest level and mean column count
        tq = encrypt_eyes(H, torch, keys, w, 999, 32, w.n_q_primes, shifts)
        tuned = H.hfe_autotune(db, tq, 0, w.d1, reps=1)
        tq.free()
    qs, p_special = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1).primes()
    n_mod = rns_moduli(w, max(list(qs) + [p_special]))
    n_b = p2_bases(w, max(list(qs) + [p_special]))
    tiles = {"rns": f"rns 256 or 128 columns per problem, {n_mod} moduli",
             "p2": f"n^2 256 or 128 columns per problem, {n_b} bases"}
    per_mac = {"i8": 50, "rns": 2 * n_mod, "p2": 2 * 3 * n_b}
    out = []
    for name in forms:
        form = codes[name]
        torch.cuda.empty_cache()
        plan = H.hfe_plan_create_for(db, items, form)
        H.hfe_plan_run(plan, items, use_graph=True)        # captures the graph
        torch.cuda.synchronize()
        same = all(np.array_equal(H.hfe_export(H.hfe_plan_result(plan, i), 0, 0, 1 << 16),
                                  H.hfe_export(H.hfe_ccmm(db, q, r0, nr, form), 0, 0, 1 << 16))
                   for i, (q, r0, nr) in list(enumerate(items))[:4])
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for _ in range(steps):
            H.hfe_plan_run(plan, items, use_graph=True)
        ev[1].record()
        torch.cuda.synchronize()
        batch_ms = (time.perf_counter() - t0) * 1e3 / steps
        dev_ms = ev[0].elapsed_time(ev[1]) / steps
        plan.free()
        seq_ms = None
        if compare_sequential:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for q, r0, nr in items:
                H.hfe_ccmm(db, q, r0, nr, form).free()
            torch.cuda.synchronize()
            seq_ms = (time.perf_counter() - t0) * 1e3
        tops = per_mac[name] * macs / (batch_ms * 1e-3) / 1e12
        res = {"form": name, "value": comparisons / (batch_ms * 1e-3), "unit": "comparisons/s",
               "ms_per_batch": batch_ms, "device_ms_per_batch": dev_ms, "int8_tops": tops,
               "frac_of_peak": tops / PEAK_I8_TOPS, "sequential_ms": seq_ms,
               "speedup_vs_sequential": (seq_ms / batch_ms) if seq_ms else None,
               "same_residues_as_single_calls": bool(same), "graph": True, "steps": steps,
               "tile": H.hfe_i8_variant_name(tuned) if name == "i8" else tiles[name],
               "items": len(mix), "columns": cols, "residue_macs": macs, "comparisons": comparisons}
        log(f"batched {name}: {batch_ms:.1f} ms per batch ({res['value']:.3e} comparisons/s, "
            f"{100 * res['frac_of_peak']:.1f}% of int8 peak), graph replay; sequential {seq_ms}")
        out.append(res)
    for q, _, _ in items:
        q.free()
    db.free()
    keys.free()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def batched_line(r, w=S.PAPER_SHARE_L5):
    return {"metric": "batched encrypted CCMM, comparisons/s (one plan: grouped launches, one persistent "
                      "contraction launch, replayed hipGraph)",
            "n_gpus": 1, "higher_is_better": True, "dtype": "i8", "data": "synthetic", **r,
            "config": {"workload": "batched_" + w.name, "items": r["items"], "eyes": "1-64", "shifts": 16,
                       "levels": "1-5 query primes + p", "rows": "2048-14336", "columns": r["columns"]}}


def run_serving(args, H, torch, rates=None, form_name=None):
    """Configuration 5: Poisson arrivals of 1-32 eyes x 16 shifts against the resident share
    database, through the continuous-batching server; throughput and arrival-to-result latency
    percentiles per arrival rate.  Returns one dict per rate.

    Queries are encrypted before the timed window (clients encrypt on their side): one ciphertext
    per eye count 1..32 serves every request of that size, so a 10 s window at 200 req/s needs
    4.3 GB of query ciphertexts rather than one per request."""
    w = S.PAPER_SHARE
    rates = rates or args.rates
    form_name = form_name or args.serve_form
    shifts = [int(x) for x in S.default_shifts(16)]
    form = {"rns": H.HFE_FORM_RNS_I8, "p2": H.HFE_FORM_P2_I8}.get(form_name, H.HFE_FORM_I8_MFMA)
    log(f"serving: encrypting the {w.d1}-code database ({form_name} form)")
    keys, db = encrypt_database(H, torch, w, form)
    dev = torch.device("cuda", 0)
    pool = {e: encrypt_eyes(H, torch, keys, w, 1000 + e, e, w.level, shifts) for e in range(1, 33)}
    torch.cuda.synchronize()
    lines = []
    for rate in rates:
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
        line = {"value": cmp / dt, "unit": "comparisons/s", "offered_req_per_s": rate, "requests": n,
                "served_req_per_s": n / dt, "seconds": dt,
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "service_p50_ms": st["service_p50_ms"],
                "service_p99_ms": st["service_p99_ms"], "steps": st["steps"],
                "mean_cols_per_step": st["mean_cols_per_step"], "max_queue": st["max_queue"],
                "rejected": st["rejected"], "max_busy_slots": st["max_busy_slots"],
                "overlap_pairs": st["overlap_pairs"], "form": form_name, "results": args.serve_results,
                "latency": ("arrival -> encrypted result ready" if encrypted else "arrival -> decrypted products"),
                "window_s": args.serve_seconds, "max_cols_per_step": args.serve_cols, "slots": 2,
                "mem_budget_gib": args.serve_budget_gib}
        log(f"serving {form_name} at {rate} req/s: served {n / dt:.1f} req/s, p50 {st['p50_ms']:.0f} ms, "
            f"p99 {st['p99_ms']:.0f} ms, {cmp / dt:.3e} comparisons/s")
        lines.append(line)
        torch.cuda.synchronize()
        for o in outs:
            if encrypted:
                o.free()
        del outs
    for q in pool.values():
        q.free()
    db.free()
    keys.free()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return lines


def serving_line(r, w=S.PAPER_SHARE):
    return {"metric": "encrypted 1:N serving, comparisons/s with continuous batching", "n_gpus": 1,
            "higher_is_better": True, "dtype": "i8", "data": "synthetic", **r,
            "config": {"workload": "serving_" + w.name, "eyes": "1-32", "shifts": 16,
                       "arrivals": f"poisson {r['offered_req_per_s']}/s", "window_s": r["window_s"],
                       "max_cols_per_step": r["max_cols_per_step"], "slots": 2,
                       "mem_budget_gib": r["mem_budget_gib"]}}


def run_lit(args, H, torch):
    """The share step at ring degree 2^16 for both layers (N_DB = N_Q = 2^16): the database is
    encrypted one prime at a time straight into its digit planes (125 GB; its 200 GB of residues are
    never resident together), then encode -> encrypt -> CCMM (int8 digits) -> decrypt -> match.
    The decrypted inner products are checked against the plaintext products of the same templates
    (ternary matrices multiplied in float32 on the device, exact below 2^24)."""
    w = S.PAPER_LIT
    work = algorithmic_work(w)
    dev = torch.device("cuda", 0)
    inp = S.make_inputs(w)
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    db_codes = torch.from_numpy(inp["db_codes"]).to(dev)
    db_masks = torch.from_numpy(inp["db_masks"]).to(dev)
    q_codes = torch.from_numpy(inp["q_codes"]).to(dev)
    q_masks = torch.from_numpy(inp["q_masks"]).to(dev)
    shifts = [int(x) for x in inp["shifts"]]
    log(f"lit: encrypting the {w.d1}-code database at N_DB = N_Q = 2^16 (digit form, one prime at a time)")
    t0 = time.perf_counter()
    m_db = H.hfe_encode(db_codes, db_masks, [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, H.HFE_FORM_I8_MFMA)
    torch.cuda.synchronize()
    t_db = time.perf_counter() - t0
    log(f"lit: database encrypted in {t_db:.2f} s ({H.hfe_db_bytes(db) / 1e9:.1f} GB of digit planes)")
    H.hfe_set_i8_variant(args.variant)
    ms_steps, kernel_ms, ip = [], [], None
    H.hfe_profile(True)
    for i in range(args.lit_steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m_q = H.hfe_encode(q_codes, q_masks, shifts)
        qct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
        r = H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_I8_MFMA)
        _, ip = H.hfe_decrypt(keys, r, v=False)
        _, eye = H.hfe_match(ip, q_masks, shifts, db_masks, want_decision=False)
        torch.cuda.synchronize()
        if i > 0:                                   # the first step warms up
            ms_steps.append((time.perf_counter() - t0) * 1e3)
            kernel_ms.append(H.hfe_profile_ms(r, 3)[1])
        r.free()
        qct.free()
    H.hfe_profile(False)
    mq = H.hfe_encode(q_codes, q_masks, shifts).float()
    ref = torch.matmul(mq, m_db.float().t().contiguous()).round().to(torch.int32)
    exact = bool(torch.equal(ref, ip))
    ms = float(np.mean(ms_steps))
    k_ms = float(np.mean(kernel_ms))
    ops = work["i8_ops"]
    line = {"metric": "encrypted query x db code comparisons/sec on 1 MI355X at ring degree 2^16",
            "value": w.d1 * w.d3 / (ms * 1e-3), "unit": "comparisons/s", "n_gpus": 1, "steps": args.lit_steps,
            "ms_per_step": ms, "higher_is_better": True, "dtype": "i8", "data": "synthetic",
            "config": {"workload": w.name, "n_db": 1 << w.log_n_db, "n_q": 1 << w.log_n_q, "query_primes": w.level,
                       "special_primes": 1, "d1": w.d1, "d2": w.d2, "d3": w.d3, "form": "i8_mfma"},
            "contraction_ms": k_ms, "int8_ops_per_launch": ops,
            "frac_of_peak": ops / (k_ms * 1e-3) / 1e12 / PEAK_I8_TOPS,
            "useful_fraction": w.d1 * w.d2 / (work["R_out"] * work["K"]),
            "db_encrypt_s": t_db, "db_digit_bytes": H.hfe_db_bytes(db),
            "ip_equals_plaintext_products": exact}
    log(f"lit: {ms:.1f} ms/step, contraction {k_ms:.1f} ms ({100 * line['frac_of_peak']:.1f}% of int8 peak); "
        f"inner products exact: {exact}")
    return line


def fs_modmuls(w: S.Workload, log_n_t: int):
    """Modular products of one FormatSwitch of the workload's queries, by kernel: ring switch
    ((level + 1) rho forward transforms of degree N_Q per ciphertext and slot, a product-accumulate of
    mask and key per coefficient, two inverse transforms with their 1/n), conversion (k (level + 1)
    forward transforms per column and slot, 1 + k products per coefficient, 1 + k inverse transforms)."""
    nq, l = 1 << w.log_n_q, w.level
    rho = 1 << (log_n_t - w.log_n_q)
    k = -(-w.d2 // nq)
    lg = w.log_n_q
    fwd, inv = nq // 2 * lg, nq // 2 * lg + nq
    ring = w.d3 * k * (l + 2) * ((l + 1) * rho * fwd + 2 * (l + 1) * rho * nq + 2 * inv)
    conv = w.d3 * (l + 2) * (k * (l + 1) * (fwd + (1 + k) * nq) + (1 + k) * inv)
    return {"ring": ring, "conv": conv, "rho": rho, "k": k}


def run_format_switch(args, H, torch, steps=5):
    """FormatSwitch (Appendix C.1) of the share workload's 512 query columns from the transmission ring
    2^16: keys, the client's transmission encryption, then `steps` timed switches (after one warm-up)
    with the stage events of the library on its stream.  The switched query goes through the CCMM
    (digit form) and must decrypt to the inner products of the same queries encrypted directly."""
    w = S.FS_SHARE
    log_n_t = S.FS_LOG_N_T[w.name]
    dev = torch.device("cuda", 0)
    inp = S.make_inputs(w)
    P = H.hfe_default_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    keys = H.hfe_keygen(P, KEY_SEED)
    t0 = time.perf_counter()
    fk = H.hfe_fs_keygen(keys, w.level, log_n_t, KEY_SEED)
    torch.cuda.synchronize()
    t_keys = time.perf_counter() - t0
    shifts = [int(x) for x in inp["shifts"]]
    m_q = H.hfe_encode(torch.from_numpy(inp["q_codes"]).to(dev), torch.from_numpy(inp["q_masks"]).to(dev), shifts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = H.hfe_fs_encrypt(fk, m_q, TX_SEED)
    torch.cuda.synchronize()
    t_tx = time.perf_counter() - t0
    log(f"format switch: keys in {t_keys:.2f} s, transmission of {w.d3} columns ({T.numel() * 8 / 1e9:.2f} GB) "
        f"in {t_tx * 1e3:.0f} ms")
    H.hfe_profile(True)
    ms, stages = [], []
    qct = None
    for i in range(steps + 1):
        if qct is not None:
            qct.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qct = H.hfe_format_switch(fk, T, w.d3)
        torch.cuda.synchronize()
        if i > 0:
            ms.append((time.perf_counter() - t0) * 1e3)
            stages.append(H.hfe_fs_profile_ms(qct, 4))
    H.hfe_profile(False)
    st = np.mean(np.array(stages), axis=0)
    m_db = H.hfe_encode(torch.from_numpy(inp["db_codes"]).to(dev), torch.from_numpy(inp["db_masks"]).to(dev), [0])
    db = H.hfe_encrypt_db(keys, m_db, DB_SEED, H.HFE_FORM_I8_MFMA)
    _, ip_fs = H.hfe_decrypt(keys, H.hfe_ccmm(db, qct, 0, w.d1, H.HFE_FORM_I8_MFMA), v=False)
    q_direct = H.hfe_encrypt(keys, m_q, w.level, Q_SEED)
    _, ip_direct = H.hfe_decrypt(keys, H.hfe_ccmm(db, q_direct, 0, w.d1, H.HFE_FORM_I8_MFMA), v=False)
    torch.cuda.synchronize()
    same = bool(torch.equal(ip_fs, ip_direct))
    mm = fs_modmuls(w, log_n_t)
    ceiling = FP64_INSTR_PER_S / FP64_PER_MODMUL
    ring_rate = mm["ring"] / (st[1] * 1e-3)
    out = {
        "workload": w.name, "n_t": 1 << log_n_t, "n_q": 1 << w.log_n_q, "rho": mm["rho"], "level": w.level,
        "transmission_primes": w.level + 1, "d2": w.d2, "d3": w.d3, "chunks_per_column": mm["k"],
        "ciphertexts": w.d3 * mm["k"], "ms": float(np.mean(ms)), "ms_min": float(np.min(ms)),
        "columns_per_s": w.d3 / (float(np.mean(ms)) * 1e-3),
        "stages_ms": {"digits": float(st[0]), "ring_switch": float(st[1]), "conversion": float(st[2]),
                      "rescales_output": float(st[3])},
        "roofline": {"bound": "alu", "kernel": "k_fs_ring", "achieved": ring_rate / 1e12,
                     "peak": ceiling / 1e12, "unit": "T modmul/s", "frac": ring_rate / ceiling,
                     "modmuls_per_launch": mm["ring"], "kernel_ms": float(st[1]), "traffic": None},
        "conversion_modmul_rate_T": mm["conv"] / (st[2] * 1e-3) / 1e12,
        "keygen_s": t_keys, "transmission_encrypt_ms": t_tx * 1e3, "transmission_bytes": T.numel() * 8,
        "ccmm_ip_equals_direct_encryption": same,
    }
    log(f"format switch: {out['ms']:.2f} ms for {w.d3} columns ({out['columns_per_s']:.0f} columns/s); stages "
        f"{', '.join(f'{k} {v:.2f}' for k, v in out['stages_ms'].items())} ms; ring switch at "
        f"{100 * out['roofline']['frac']:.1f}% of the modular-product ceiling; CCMM equals direct: {same}")
    return out


# f(x) = sum_j c_j x^j, the folding polynomial of Appendix C.2 (to check the decrypted fold)
FOLD_COEFFS = (0.004105, -0.173510, -2.528271, 24.347349, 124.161550, -412.746212, 376.961251, 106.553952)


def fold_expected(w: S.FoldWorkload, ip: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """The values the folded ciphertexts must decrypt to: per group, sum_r' roll(f(ip / count), r k + r')."""
    slots = ip.shape[1]
    f = np.polyval(np.array(FOLD_COEFFS[::-1]), ip.astype(np.float64) / counts)
    out = []
    for b in range(w.blocks):
        for r in range(-(-w.rho // w.k)):
            acc = np.zeros(slots)
            for rp in range(min(w.k, w.rho - r * w.k)):
                acc += np.roll(f[b * w.rho + r * w.k + rp], r * w.k + rp)
            out.append(acc)
    return np.array(out)


def fold_modmuls(w: S.FoldWorkload):
    """Modular products of the f stage of one fold (all ciphertexts), counted from its operations: a
    transform of degree N is N/2 log N butterflies of one product (an inverse adds N for its 1/N).
    A product of ciphertexts at level l: the tensor's a_x a_y and the digit factor on l + 1 inverse
    transforms, (l + 1)^2 forward transforms of the digits (none at a digit's own prime, where the tensor
    and the factor are taken again: two products per coefficient), two key products per coefficient for
    each of the (l + 2)(l + 1) digit and prime pairs, two inverse transforms at p; rescaled, the sums and p (d0, d1) are divided by p q_l in one rounding: two
    inverse transforms at q_l with the tensor at q_l, p d and the CRT (7 products per coefficient over both
    parts), and 2 l forward transforms with (p q_l)^-1, the tensor and q_l^-1 (7 per coefficient and slot over
    both parts); unrescaled, 2 (l + 1) forward transforms with p^-1 and the tensor (5 per coefficient and
    slot).  The constant terms share two inverse transforms of x's last slot (k x_3 transforms to k u); each,
    rescaled from level 3 to `to`, takes k u (2 products per coefficient) and 2 (to + 1) forward transforms
    with two products per coefficient."""
    n, lg = 1 << w.log_n, w.log_n
    fwd, inv = n // 2 * lg, n // 2 * lg + n

    def mul(l, rescaled=True):
        sums = (l + 1) * (inv + 2 * n) + (l + 1) ** 2 * fwd + (l + 2) * (l + 1) * 2 * n + (l + 1) * 2 * n + 2 * inv
        if rescaled:
            return sums + 2 * inv + 7 * n + 2 * l * fwd + 7 * l * n
        return sums + 2 * (l + 1) * fwd + 5 * (l + 1) * n

    def const(to):
        return 2 * n + 2 * (to + 1) * (fwd + 2 * n)

    f = mul(3) + 2 * inv + const(2) + const(2) + const(1) + const(1) + 3 * mul(2) + mul(1, rescaled=False)
    return w.count * f


def run_fold(args, H, torch, steps=3):
    """Normalise and fold (Algorithm 2 after the CCMM) of the share workload's scores: 512 query columns
    against 14,336 database entries, two blocks of 8,192 slots at ring degree 2^14, k = 16.  Keys and
    the encryption of the inner products first (untimed), then `steps` timed folds after one warm-up with
    the library's stage events.  The folded ciphertexts are decrypted on the GPU and checked against the
    plain folded values."""
    w = S.FOLD_SHARE
    ip, counts = S.fold_inputs(w)
    t0 = time.perf_counter()
    fk = H.hfe_fold_keygen(w.log_n, w.k, w.rho, KEY_SEED)
    torch.cuda.synchronize()
    t_keys = time.perf_counter() - t0
    ip_d, cnt_d = torch.from_numpy(ip).cuda(), torch.from_numpy(counts).cuda()
    t0 = time.perf_counter()
    ct = H.hfe_fold_encrypt(fk, ip_d, FOLD_SEED)
    torch.cuda.synchronize()
    t_enc = time.perf_counter() - t0
    log(f"fold: keys in {t_keys:.2f} s, {w.count} score ciphertexts encrypted in {t_enc * 1e3:.0f} ms")
    H.hfe_profile(True)
    ms, stages = [], []
    out = None
    for i in range(steps + 1):
        if out is not None:
            out.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = H.hfe_fold(fk, ct, cnt_d, w.rho)
        torch.cuda.synchronize()
        if i > 0:
            ms.append((time.perf_counter() - t0) * 1e3)
            stages.append(H.hfe_fold_profile_ms(out, 4))
    H.hfe_profile(False)
    st = np.mean(np.array(stages), axis=0)
    vals = H.hfe_fold_decrypt(fk, out).cpu().numpy()
    err = float(np.max(np.abs(vals - fold_expected(w, ip, counts))))
    groups = w.blocks * -(-w.rho // w.k)
    mean = float(np.mean(ms))
    res = {
        "workload": w.name, "n": 1 << w.log_n, "k": w.k, "rho": w.rho, "blocks": w.blocks, "d1": w.d1,
        "ciphertexts": w.count, "folded_ciphertexts": groups, "slots": w.count * (1 << w.log_n) // 2,
        "ms": mean, "ms_min": float(np.min(ms)), "ciphertexts_per_s": w.count / (mean * 1e-3),
        "scores_per_s": w.d1 * (w.count // w.blocks) / (mean * 1e-3),
        "stages_ms": {"mu_plaintexts": float(st[0]), "normalise": float(st[1]), "f": float(st[2]),
                      "rotations_sums": float(st[3])},
        "keygen_s": t_keys, "encrypt_ms": t_enc * 1e3, "max_abs_error_vs_plain": err,
    }
    mm = fold_modmuls(w)
    ceiling = FP64_INSTR_PER_S / FP64_PER_MODMUL
    rate = mm / (st[2] * 1e-3)
    res["roofline"] = {"bound": "alu", "kernel": "f stage (k_fold_ks_mac, k_fold_lift, k_fold_inv, element-wise passes)",
                       "achieved": rate / 1e12, "peak": ceiling / 1e12, "unit": "T modmul/s", "frac": rate / ceiling,
                       "modmuls_per_launch": mm, "kernel_ms": float(st[2]), "traffic": None}
    log(f"fold: {mean:.2f} ms for {w.count} ciphertexts ({res['ciphertexts_per_s']:.0f} ciphertexts/s); stages "
        f"{', '.join(f'{k} {v:.2f}' for k, v in res['stages_ms'].items())} ms; max error vs plain {err:.2e}; "
        f"f stage at {100 * res['roofline']['frac']:.1f}% of the modular-product ceiling")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--workload", default=S.PAPER_SHARE.name, choices=sorted(S.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle baseline processes (0: the host's CPUs, at most 16)")
    ap.add_argument("--cpu-rows", type=int, default=1024, help="oracle baseline: database rows per process (power of 2)")
    ap.add_argument("--cpu-cols", type=int, default=32, help="oracle baseline: query columns of the CCMM sample")
    ap.add_argument("--sweep", action="store_true", help="time every int8 tile configuration and exit")
    ap.add_argument("--variant", type=int, default=-1, help="int8 tile configuration (-1: default)")
    ap.add_argument("--ccmm-only", type=int, default=0, help="run N int8 CCMMs after setup and exit (profiling)")
    ap.add_argument("--form", choices=("i8", "rns", "p2", "chain"), default="i8",
                    help="with --ccmm-only: the int8 form to run (chain: the n^2 modulus chain)")
    ap.add_argument("--lit-steps", type=int, default=3, help="lit mode: timed steps")
    ap.add_argument("--chain-q-mods", type=int, default=7, help="n^2 chain: query moduli (3 more form P)")
    ap.add_argument("--no-fs", action="store_true", help="step mode: skip FormatSwitch")
    ap.add_argument("--fs-steps", type=int, default=5, help="FormatSwitch: timed switches")
    ap.add_argument("--no-fold", action="store_true", help="step mode: skip normalise and fold")
    ap.add_argument("--fold-steps", type=int, default=3, help="fold: timed folds")
    ap.add_argument("--mode", choices=("step", "batched", "serving", "lit", "fs", "fold"), default="step",
                    help="step: the hot-path step (default); batched: 64 uneven items as one plan; "
                         "serving: Poisson arrivals through the server; lit: the step at N_DB = N_Q = 2^16")
    ap.add_argument("--batch-items", type=int, default=64)
    ap.add_argument("--batched-steps", type=int, default=3, help="step mode: timed replays of the batch")
    ap.add_argument("--no-batched", action="store_true", help="step mode: skip the batched configuration")
    ap.add_argument("--no-serving", action="store_true", help="step mode: skip the serving configuration")
    ap.add_argument("--default-rates", type=float, nargs="+", default=[200.0, 50.0],
                    help="step mode: serving arrival rates, req/s")
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

    w = S.WORKLOADS[args.workload]
    work = algorithmic_work(w)
    inp = S.make_inputs(w)
    cpu = cpu_chain = cpu_fs = cpu_fold = None
    if args.mode == "step" and not args.no_cpu_baseline and not (args.sweep or args.ccmm_only):
        # before anything touches the GPU: the oracle's process pool is forked from this process
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        log(f"timing the oracle on a bounded sample ({workers} processes)")
        cpu = cpu_baseline(w, inp, workers, args.cpu_rows, args.cpu_cols, enc_cols=4, dec_rows=1024)
        log(f"oracle: {cpu['sample']}")
        cpu.pop("step_s")
        if w.name == S.PAPER_SHARE.name:
            cpu_chain, cpu_fs, cpu_fold = cpu_baseline_chain_fs(w, inp, args.chain_q_mods)
            log(f"oracle: {cpu_chain['sample']}")
            log(f"oracle: {cpu_fs['sample']}")
            log(f"oracle: {cpu_fold['sample']}")

    import torch
    import paper_2601_17561_amd as H

    if args.mode == "batched":
        for r in run_batched(args, H, torch):
            print(json.dumps(batched_line(r)), flush=True)
        return
    if args.mode == "serving":
        for r in run_serving(args, H, torch):
            print(json.dumps(serving_line(r)), flush=True)
        return
    if args.mode == "lit":
        print(json.dumps(run_lit(args, H, torch)), flush=True)
        return
    if args.mode == "fold":
        print(json.dumps(run_fold(args, H, torch, steps=args.fold_steps)), flush=True)
        return
    if args.mode == "fs":
        print(json.dumps(run_format_switch(args, H, torch, steps=args.fs_steps)), flush=True)
        if args.copy_mib:  # a plain device copy of known size (counter calibration)
            src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            log(f"copied {args.copy_mib} MiB")
        return
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    log(f"workload {w.name}: d1={w.d1} d2={w.d2} d3={w.d3} N_DB=2^{w.log_n_db} N_Q=2^{w.log_n_q} "
        f"primes={w.level}+p")
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

    chain_kd = {}
    # the paper's own modulus chain (Section 6.3): query moduli n^2 for the largest primes n <= 253 (as
    # many as give Q about the bits of the level's 36-bit primes), 3 more for P; the same secrets
    chain_q = args.chain_q_mods
    Cp = H.hfe_chain_default_params(w.log_n_db, w.log_n_q, chain_q, 3, w.d2, w.d1)
    chain_kd["keys"] = H.hfe_chain_keygen(Cp, KEY_SEED)
    chain_kd["level"] = chain_q
    m_db = H.hfe_encode(db_codes, db_masks, [0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain_kd["db"] = H.hfe_encrypt_db(chain_kd["keys"], m_db, DB_SEED, H.HFE_FORM_P2_I8)
    torch.cuda.synchronize()
    t_chain_db = time.perf_counter() - t0
    del m_db
    log(f"n^2 chain: {chain_q} query moduli + 3 special ({Cp.q_bases()} | {Cp.p_bases()}), database in "
        f"{t_chain_db:.2f} s")

    def step(form, profile_out=None, marks=None):
        # marks: 6 events recorded on the stream the library runs on (torch's current stream)
        # around encode, encrypt, CCMM, decrypt and match
        mark = (lambda i: marks[i].record()) if marks is not None else (lambda i: None)
        k_, db_, lvl = (chain_kd["keys"], chain_kd["db"], chain_kd["level"]) if form == "chain" else (keys, db, w.level)
        mark(0)
        m_q = H.hfe_encode(q_codes, q_masks, shifts)
        mark(1)
        qct = H.hfe_encrypt(k_, m_q, lvl, Q_SEED)
        mark(2)
        r = H.hfe_ccmm(db_, qct, 0, w.d1, H.HFE_FORM_P2_I8 if form == "chain" else form)
        mark(3)
        _, ip = H.hfe_decrypt(k_, r, v=False)
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
        db_ = db
        if args.form == "chain":
            qct = H.hfe_encrypt(chain_kd["keys"], m_q, chain_kd["level"], Q_SEED)
            form, db_ = H.HFE_FORM_P2_I8, chain_kd["db"]
        for _ in range(args.ccmm_only):
            H.hfe_ccmm(db_, qct, 0, w.d1, form).free()
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
                                    ("chain", "chain", args.steps, args.warmup),
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
    same_chain = bool(torch.equal(results["chain"]["ip"], results["i8"]["ip"]))
    chain_slots = chain_q + 3
    chain_ops = 2 * 3 * chain_slots * work["R_out"] * work["K"] * w.d3
    import math
    chain_q_bits = sum(2 * math.log2(n) for n in Cp.q_bases())
    chain_p_bits = sum(2 * math.log2(n) for n in Cp.p_bases())
    # measured instruction ceilings on this device: int8 MFMA on streaming random operands (the
    # digit planes of ciphertexts are uniformly random) and on zero operands, and the VALU
    # 32 x 32 -> 64-bit multiply-add the plain form spends four of per residue multiply-add
    rates = {"mfma_i8_random_tops": max(H.hfe_probe_rate(H.HFE_PROBE_MFMA_I8, 2000) for _ in range(3)) / 1e12,
             "mfma_i8_zero_tops": max(H.hfe_probe_rate(H.HFE_PROBE_MFMA_I8_ZERO, 2000) for _ in range(3)) / 1e12,
             "valu_mad_u64_per_s": max(H.hfe_probe_rate(H.HFE_PROBE_VALU_MAD_U64, 4000) for _ in range(3))}
    log(f"ceilings: int8 MFMA {rates['mfma_i8_random_tops']:.0f} TOP/s on random operands, "
        f"{rates['mfma_i8_zero_tops']:.0f} on zeros; v_mad_u64_u32 {rates['valu_mad_u64_per_s']:.3e}/s")

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
                     "kernel_ms": i8["contraction_ms"],
                     "measured_ceiling": rates["mfma_i8_random_tops"],
                     "frac_of_measured_ceiling": achieved / rates["mfma_i8_random_tops"]},
        "ceilings": rates,
        "plain": ({"ms_per_step": plain["ms_per_step"],
                   "comparisons_per_s": plain["comparisons_per_s"],
                   "contraction_ms": plain["contraction_ms"],
                   "residue_macs_per_s": work["residue_macs"] / (plain["contraction_ms"] * 1e-3),
                   "roofline": {"bound": "alu", "unit": "residue multiply-adds/s",
                                "achieved": work["residue_macs"] / (plain["contraction_ms"] * 1e-3),
                                "peak": rates["valu_mad_u64_per_s"] / 4,
                                "frac": work["residue_macs"] / (plain["contraction_ms"] * 1e-3)
                                / (rates["valu_mad_u64_per_s"] / 4),
                                "basis": "4 v_mad_u64_u32 per residue multiply-add (18-bit limbs), "
                                         "measured instruction rate"}}
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
        "chain": {"form": f"the paper's n^2 modulus chain: {chain_q} query moduli n^2 ({Cp.q_bases()}), P of 3 "
                          f"({Cp.p_bases()}), 3 int8 products per modulus, no integer rebuilt",
                  "ms_per_step": results["chain"]["ms_per_step"],
                  "comparisons_per_s": results["chain"]["comparisons_per_s"],
                  "contraction_ms": results["chain"]["contraction_ms"], "lift_ms": results["chain"]["lift_ms"],
                  "rescale_ms": results["chain"]["rescale_ms"],
                  "int8_ops_per_launch": chain_ops,
                  "frac_of_peak": chain_ops / (results["chain"]["contraction_ms"] * 1e-3) / 1e12 / PEAK_I8_TOPS,
                  "Q_bits": chain_q_bits, "P_bits": chain_p_bits, "db_encrypt_s": t_chain_db,
                  "over_i8_step": i8["ms_per_step"] / results["chain"]["ms_per_step"],
                  "over_rns_step": rns["ms_per_step"] / results["chain"]["ms_per_step"],
                  "equals_i8_ip": same_chain, "phases_ms": results["chain"]["phases_ms"],
                  "cpu_baseline": cpu_chain},
        "i8_over_plain_step": plain["ms_per_step"] / i8["ms_per_step"] if plain else None,
        "stages_ms": {"lift_split": i8["lift_ms"], "contraction": i8["contraction_ms"],
                      "contraction_median": i8["contraction_median_ms"], "rescale": i8["rescale_ms"]},
        "phases_ms": i8["phases_ms"],
        "i8_equals_plain_ip": same,
        "db_encrypt_s": t_db,
        "cpu_baseline": cpu,
    }
    # configurations 4 and 5 on the same device, after the share databases are released
    del db, prof
    chain_kd.pop("db")
    chain_kd.clear()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_batched:
        line["batched"] = run_batched(args, H, torch, forms=("i8", "rns"), steps=args.batched_steps,
                                      compare_sequential=False)
    if not args.no_serving:
        line["serving"] = run_serving(args, H, torch, rates=args.default_rates, form_name="rns")
    if not args.no_fs:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        line["format_switch"] = run_format_switch(args, H, torch, steps=args.fs_steps)
        line["format_switch"]["cpu_baseline"] = cpu_fs
    if not args.no_fold:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        line["fold"] = run_fold(args, H, torch, steps=args.fold_steps)
        line["fold"]["cpu_baseline"] = cpu_fold
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
