"""Writes share_samples.json: oracle values of sampled entries of the share workload.

The share workload (N_DB = 2^14, N_Q = 2^13, three query primes plus p, 14,336 database codes of
12,800 bits, 32 eyes x 16 shifts = 512 query columns) is too large for the full-matrix oracle.  This
script evaluates, with the oracle only (oracle/ and the seeded templates of hfe_synth):

  * result residues of a grid of output entries: 32 output rows (16 A-part rows, 16 database codes
    including the first and last) x 64 query columns (8 in every 64-column tile, both ends of each
    tile among them) x 3 query primes = 6,144 residues, each RS_p of the exact product of a whole
    database row with the lifted query column (ckks.ccmm_entries);
  * database ciphertext entries: the same 32 rows at 32 columns (both ends of each block of K) for
    each of the 4 primes = 4,096 residues (ckks.db_rows).

Run from the repository root:  python tests/golden/make_share_samples.py
The seeds are those of tests/test_gpu_scale.py (keys 41, database 42, query 43).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import hfe_synth as S  # noqa: E402
from oracle import ckks as OC  # noqa: E402
from oracle import iris as OI  # noqa: E402
from oracle import params as OP  # noqa: E402

KEY_SEED, DB_SEED, Q_SEED = 41, 42, 43
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "share_samples.json")


def sample_rows(P, d1, g):
    a = [0, 1, 63, 64, 127, 128, 255, 256, P.n_db // 2 - 1, P.n_db // 2, P.n_db - 1]
    a += sorted(set(g.integers(0, P.n_db, 16).tolist()) - set(a))[:16 - len(a)]
    b = [0, 1, 63, 64, 127, 128, d1 // 2, d1 - 1]
    b += sorted(set(g.integers(0, d1, 16).tolist()) - set(b))[:16 - len(b)]
    return sorted(a) + [P.n_db + x for x in sorted(b)]


def sample_cols(d3, g):
    cols = []
    for t0 in range(0, d3, 64):
        c = {t0, t0 + 63}
        while len(c) < 8:
            c.add(int(g.integers(t0, t0 + 64)))
        cols += sorted(c)
    return cols


def main():
    t0 = time.time()
    w = S.PAPER_SHARE
    P = OP.make_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)
    inp = S.make_inputs(w)
    keys = OC.keygen(P, KEY_SEED)
    m_db = OI.ternary(inp["db_codes"], inp["db_masks"])
    qc, qm = OI.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    m_q = OI.ternary(qc, qm)
    g = np.random.default_rng(20260117)
    rows = sample_rows(P, w.d1, g)
    cols = sample_cols(w.d3, g)
    kcols = sorted({0, 1, 63, 64, P.d2 - 1, P.d2, P.K - 64, P.K - 1} |
                   set(g.integers(0, P.K, 40).tolist()))[:32]
    ids = OC.prime_ids(P, len(P.q))
    d_rows = {}
    for pid, prime in ids:
        print(f"database rows, prime {prime} ({time.time() - t0:.0f} s)", flush=True)
        d_rows[pid] = OC.db_rows(keys, m_db, DB_SEED, pid, prime, rows)
    print(f"query columns ({time.time() - t0:.0f} s)", flush=True)
    xt = OC.query_columns(keys, m_q[cols], cols, w.level, Q_SEED)
    print(f"result entries ({time.time() - t0:.0f} s)", flush=True)
    res = OC.ccmm_entries(P, {pid: d_rows[pid] for pid, _ in OC.prime_ids(P, w.level)}, xt, w.level)
    doc = {
        "about": "oracle values of sampled entries of the share workload; written by make_share_samples.py",
        "workload": w.name,
        "seeds": {"keys": KEY_SEED, "db": DB_SEED, "query": Q_SEED},
        "rows": rows,
        "cols": cols,
        "result": [res[i].tolist() for i in range(w.level)],          # [prime i][col][row]
        "db_cols": kcols,
        "db": [d_rows[pid][:, kcols].tolist() for pid, _ in ids],      # [prime slot][row][k]
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
