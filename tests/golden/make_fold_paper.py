"""Writes fold_paper.json: the oracle's normalise-and-fold at the fold's largest ring degree (2^14).

The FOLD_PAPER workload (N = 2^14, k = 16 as in Appendix C.2, one block of 16 score ciphertexts, mask
counts of 12,800-bit codes) runs oracle.fold end to end with the seeds of tests/test_gpu_fold.py
(keys 101, input encryption 707: tests/oracle_cases.py).  The arrays are too large to store, so the
file keeps the SHA-256 of each in the library's export order as little-endian int64 (the secret, the
input ciphertexts and the folded ciphertexts, each [count][b | a][q_0 .. q_level][N] coefficient
residues), and sampled entries that name the first differing ones when a hash does not match.

Run from the repository root:  python tests/golden/make_fold_paper.py
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
from oracle_cases import fold_case, fold_layout  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fold_paper.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def samples(a: np.ndarray, n: int, g) -> dict:
    flat = a.reshape(-1)
    idx = np.unique(np.concatenate([[0, flat.size - 1], g.integers(0, flat.size, n)]))
    return {"index": idx.tolist(), "value": flat[idx].tolist()}


def main():
    t0 = time.time()
    w = S.FOLD_PAPER
    c = fold_case(w.name)
    arr = dict(s=c.keys.s.astype(np.int64), ct=fold_layout(c.P, c.cts), out=fold_layout(c.P, c.out))
    g = np.random.default_rng(w.seed)
    res = {w.name: {
        "shapes": {k: list(v.shape) for k, v in arr.items()},
        "sha256": {k: digest(v) for k, v in arr.items()},
        "samples": {k: samples(arr[k], 1024, g) for k in ("ct", "out")},
    }}
    with open(OUT, "w") as f:
        json.dump(res, f)
    print(f"{w.name}: {time.time() - t0:.1f} s; wrote {OUT}")


if __name__ == "__main__":
    main()
