"""Writes big_ring.json: the oracle's results for the two ring-degree-2^16 workloads.

BIG_DB (N_DB = 2^16, N_Q = 2^9) and BIG_Q (N_DB = 2^9, N_Q = 2^16) each run the full oracle
(keys, database and query encryption, CCMM, decryption) with the seeds of tests/test_gpu_big_ring.py
(keys 101, database 202, query 303: tests/oracle_cases.py).  The arrays are too large to store, so the
file keeps, per workload:
  * the SHA-256 of every residue array in the library's canonical export order, as little-endian
    int64: the query secrets, the database secrets, the database D ([prime][column][row]), the query
    ciphertext ([prime][column][b | a]) and the CCMM result ([prime][column][A_out | B_out]);
  * sampled entries of the database, the query and the result (indices and values), which name the
    first differing entries when a hash does not match;
  * the decrypted inner products (d3 x d1) of the oracle.
A GPU test that reproduces every hash has reproduced every residue of these arrays.

Run from the repository root:  python tests/golden/make_big_ring.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import hfe_synth as S  # noqa: E402
from oracle_cases import case  # noqa: E402
from oracle import prng  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "big_ring.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def canonical(c):
    """The oracle's arrays in the library's export order."""
    w, P = c.w, c.P
    all_ids = [i for i in range(len(P.q))] + [prng.P_ID]
    D = np.stack([c.D[pid].T for pid in all_ids])                    # [prime][col][row]
    XT = np.stack([c.XT[i] for i in range(w.level)])                  # [prime][col][K]
    out = np.stack([c.out[i] for i in range(w.level)])                # [prime][col][R_out]
    return dict(s_q=c.keys.s.astype(np.int64), s_db=c.keys.s_db.astype(np.int64), D=D, XT=XT, out=out)


def samples(a: np.ndarray, n: int, g) -> dict:
    flat = a.reshape(-1)
    idx = np.unique(np.concatenate([[0, flat.size - 1], g.integers(0, flat.size, n)]))
    return {"index": idx.tolist(), "value": flat[idx].tolist()}


def main():
    res = {}
    for w in (S.BIG_DB, S.BIG_Q):
        t0 = time.time()
        c = case(w.name)
        arr = canonical(c)
        g = np.random.default_rng(w.seed)
        assert np.array_equal(c.ip, c.ip_true), "oracle decryption differs from the popcount truth"
        res[w.name] = {
            "shapes": {k: list(v.shape) for k, v in arr.items()},
            "sha256": {k: digest(v) for k, v in arr.items()},
            "samples": {k: samples(arr[k], 512, g) for k in ("D", "XT", "out")},
            "ip": c.ip.tolist(),
        }
        print(f"{w.name}: {time.time() - t0:.1f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
