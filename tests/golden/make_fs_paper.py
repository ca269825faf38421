"""Writes fs_paper.json: the oracle's FormatSwitch at the paper's ring degrees (2^16 -> 2^13).

The FS_PAPER workload (12,800-bit codes, CCMM level 3, transmission modulo four primes, two query
columns) runs oracle.formatswitch end to end with the seeds of tests/test_gpu_fswitch.py (keys 101,
transmission 404: tests/oracle_cases.py).  The arrays are too large to store, so the file keeps the
SHA-256 of each in the library's export order as little-endian int64 (the secrets s_T and s', the
transmission ciphertexts [prime][column][a | b][N_T], the switched query [prime][column][b | a]),
sampled entries that name the first differing ones when a hash does not match, and the popcount
truth of the queries against the workload's database codes.

Run from the repository root:  python tests/golden/make_fs_paper.py
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
from oracle_cases import fs_case  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fs_paper.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def samples(a: np.ndarray, n: int, g) -> dict:
    flat = a.reshape(-1)
    idx = np.unique(np.concatenate([[0, flat.size - 1], g.integers(0, flat.size, n)]))
    return {"index": idx.tolist(), "value": flat[idx].tolist()}


def main():
    t0 = time.time()
    w = S.FS_PAPER
    c = fs_case(w.name)
    arr = dict(s_t=c.F.s_t.astype(np.int64), s_r=c.F.s_r.astype(np.int64), T=c.T, XT=c.XT)
    g = np.random.default_rng(w.seed)
    res = {w.name: {
        "log_n_t": c.log_n_t,
        "shapes": {k: list(v.shape) for k, v in arr.items()},
        "sha256": {k: digest(v) for k, v in arr.items()},
        "samples": {k: samples(arr[k], 1024, g) for k in ("T", "XT")},
        "ip_true": c.ip_true.tolist(),
    }}
    with open(OUT, "w") as f:
        json.dump(res, f)
    print(f"{w.name}: {time.time() - t0:.1f} s; wrote {OUT}")


if __name__ == "__main__":
    main()
