"""Writes fold_paper.json: the oracle's normalise-and-fold at the fold's largest ring degree (2^14).

Two cases, both with the seeds of tests/test_gpu_fold.py (keys 101, input encryption 707:
tests/oracle_cases.py):
* the FOLD_PAPER workload (N = 2^14, k = 16 as in Appendix C.2, one block of 16 score ciphertexts, mask
  counts of 12,800-bit codes), end to end;
* the first two groups of the share workload's fold (FOLD_SHARE: blocks of 512, 1,024 ciphertexts): they
  depend only on the first 32 score ciphertexts and use the rotation keys 1 .. 15 and 16, which the keys
  of blocks of 32 number as the keys of blocks of 512 do, so the oracle folds those 32 ciphertexts in a
  block of 32 and the library's full-size fold must give the same first two ciphertexts.
The arrays are too large to store, so the file keeps the SHA-256 of each in the library's export order as
little-endian int64 (the secret, the input ciphertexts and the folded ciphertexts, each [count][b | a]
[q_0 .. q_level][N] coefficient residues), and sampled entries that name the first differing ones when a
hash does not match.

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


SHARE_HEAD = 32   # ciphertexts of the share workload's first two groups


def share_head():
    """The oracle's fold of the share workload's first 32 score ciphertexts in a block of 32."""
    from oracle import fold as OF
    from oracle_cases import FOLD_SEED, KEY_SEED
    w = S.FOLD_SHARE
    P = OF.fold_params(w.log_n, w.k)
    keys = OF.fold_keygen(P, KEY_SEED, OF.rot_amounts(w.k, SHARE_HEAD))
    ip, counts = S.fold_inputs(w)
    cts = [OF.encrypt(keys, ip[c].astype(np.int64), FOLD_SEED, c) for c in range(SHARE_HEAD)]
    out = OF.fold(keys, cts, counts[:SHARE_HEAD].astype(np.int64), SHARE_HEAD)
    return P, out


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
    print(f"{w.name}: {time.time() - t0:.1f} s")
    P, out = share_head()
    head = fold_layout(P, out)
    res[S.FOLD_SHARE.name + "_head"] = {
        "shapes": {"out": list(head.shape)},
        "sha256": {"out": digest(head)},
        "samples": {"out": samples(head, 1024, g)},
    }
    with open(OUT, "w") as f:
        json.dump(res, f)
    print(f"share head: {time.time() - t0:.1f} s; wrote {OUT}")


if __name__ == "__main__":
    main()
