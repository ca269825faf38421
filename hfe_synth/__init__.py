"""Seeded synthetic iris templates for the encrypted 1:N matching workloads.

This module produces raw template bits only: iris codes, masks, the cyclic
shift offsets applied to query eyes, and planted near-copies of database rows
(so that match decisions are exercised).  It holds none of the encryption,
encoding or matching arithmetic; both the HIP library's callers and the CPU
oracle take their inputs from here.

Template model (Section 2.1 of the paper: code c and mask m are bit vectors of
the same length):
  * code bits   ~ i.i.d. Bernoulli(p_code)   (0.5 by default)
  * mask bits   ~ i.i.d. Bernoulli(p_mask)   (0.9 by default)
  * a planted query eye is a database row whose code bits are flipped with
    probability `flip`, then cyclically rotated by -r* so that the query column
    with shift r* realigns it with the database row.

Every array is numpy uint8 holding 0/1, row-major (one template per row).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 260117561


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def db_templates(seed: int, d1: int, d2: int, p_code: float = 0.5,
                 p_mask: float = 0.9) -> Tuple[np.ndarray, np.ndarray]:
    """Return (codes, masks), each uint8 of shape (d1, d2) with 0/1 entries."""
    g = _rng(seed, 1)
    codes = (g.random((d1, d2)) < p_code).astype(np.uint8)
    masks = (g.random((d1, d2)) < p_mask).astype(np.uint8)
    return codes, masks


@dataclasses.dataclass(frozen=True)
class Planted:
    eye: int        # query eye index
    db_row: int     # database row it is a noisy copy of
    shift: int      # r*: the query column with this shift realigns the copy
    flip: float     # probability of flipping each code bit


def query_eyes(seed: int, n_eyes: int, d2: int, db_codes: np.ndarray,
               db_masks: np.ndarray, planted: Sequence[Planted] = (),
               p_code: float = 0.5, p_mask: float = 0.9
               ) -> Tuple[np.ndarray, np.ndarray]:
    """Return (codes, masks) of shape (n_eyes, d2) for the query eyes.

    Eyes not listed in `planted` are fresh random templates.  A planted eye is
    roll(noisy copy of db row, -shift) for code and mask alike (rotation moves
    code and mask together, Section 2.1.2 of the paper).
    """
    g = _rng(seed, 2)
    codes = (g.random((n_eyes, d2)) < p_code).astype(np.uint8)
    masks = (g.random((n_eyes, d2)) < p_mask).astype(np.uint8)
    for pl in planted:
        gp = _rng(seed, 1000 + pl.eye)
        flips = (gp.random(d2) < pl.flip).astype(np.uint8)
        c = db_codes[pl.db_row] ^ flips
        m = db_masks[pl.db_row].copy()
        codes[pl.eye] = np.roll(c, -pl.shift)
        masks[pl.eye] = np.roll(m, -pl.shift)
    return codes, masks


def default_shifts(n_shifts: int) -> np.ndarray:
    """Shift offsets r for the query columns: {-n/2, ..., n/2-1}; [0] if n == 1."""
    if n_shifts == 1:
        return np.zeros(1, dtype=np.int32)
    return np.arange(-(n_shifts // 2), n_shifts - n_shifts // 2, dtype=np.int32)


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shapes of one synthetic workload (ring degrees, primes, template sizes)."""
    name: str
    log_n_db: int
    log_n_q: int
    n_q_primes: int        # query primes the database carries
    level: int             # query primes used by the query (l_Q)
    d1: int                # database codes
    d2: int                # code length in bits
    eyes: int              # query eyes
    n_shifts: int          # cyclic shifts per eye (query columns = eyes * n_shifts)
    planted: Tuple[Planted, ...] = ()
    seed: int = BASE_SEED

    @property
    def d3(self) -> int:
        return self.eyes * self.n_shifts


def _planted(eyes: int, d1: int, n_shifts: int, count: int, seed: int) -> Tuple[Planted, ...]:
    g = _rng(seed, 3)
    out = []
    sh = default_shifts(n_shifts)
    eye_ids = g.choice(eyes, size=min(count, eyes), replace=False)
    for e in sorted(int(x) for x in eye_ids):
        out.append(Planted(eye=e, db_row=int(g.integers(0, d1)),
                           shift=int(sh[int(g.integers(0, len(sh)))]), flip=0.1))
    return tuple(out)


# Tiny plain workload: N = 2^12 for both layers, one query prime plus the
# special prime, 4 query codes against 256 database codes of 1024 bits; query 0
# is a planted copy of database row 17.
TINY = Workload("tiny_n4096_d1_256_d2_1024_q4", 12, 12, 1, 1, 256, 1024, 4, 1,
                planted=(Planted(0, 17, 0, 0.1),), seed=BASE_SEED + 1)

# Small multi-chunk workload: several secrets per layer (k = 2, k' = 2).
TINY_MULTI = Workload("tinymulti_ndb128_nq512_d1_256_d2_1024_q4", 7, 9, 2, 2, 256, 1024, 2, 2,
                      planted=(Planted(1, 200, -1, 0.1),), seed=BASE_SEED + 11)

# Mid-size workload whose shapes cross every tile boundary of the contraction kernels: 956 output
# rows (256 A rows + 700 codes: ragged against 64-, 128- and 256-row tiles), 272 query columns
# (17 eyes x 16 shifts: two 128-column tiles plus 16, one 256-column tile plus 16), three chunks
# per secret stack (d2 = 1280 over N_Q = 512, the last one truncated; 700 codes over N_DB = 256),
# three query primes plus the special prime.
MID = Workload("mid_ndb256_nq512_L3p_d1_700_d2_1280_q272", 8, 9, 3, 3, 700, 1280, 17, 16,
               seed=BASE_SEED + 21)

# One GPU's share at paper scale: N_DB = 2^14, N_Q = 2^13, three query primes
# plus the special prime, 32 eyes x 16 shifts = 512 query columns against
# 14,336 database codes of 12,800 bits.
PAPER_SHARE = Workload("share_ndb16384_nq8192_L3p_d1_14336_d2_12800_q512", 14, 13, 3, 3,
                       14336, 12800, 32, 16, seed=BASE_SEED + 2)



# Ring degree 2^16 (the transmission ring of Appendix C.1), one layer at a time so that the
# oracle stays tractable: a database layer of N_DB = 2^16 with a small query layer, and a query
# layer of N_Q = 2^16 with a small database layer; one query prime plus p, 256 codes of 1024 bits,
# 4 query columns (query 0 a planted copy of database row 17).
BIG_DB = Workload("bigdb_ndb65536_nq512_L1p_d1_256_d2_1024_q4", 16, 9, 1, 1, 256, 1024, 4, 1,
                  planted=(Planted(0, 17, 0, 0.1),), seed=BASE_SEED + 31)
BIG_Q = Workload("bigq_ndb512_nq65536_L1p_d1_256_d2_1024_q4", 9, 16, 1, 1, 256, 1024, 4, 1,
                 planted=(Planted(0, 17, 0, 0.1),), seed=BASE_SEED + 32)

# Workloads of the n^2 modulus chain (Section 6.3): n_q_primes counts the query moduli n^2 (the
# special part has 3 more).  Tiny: rings of 2^9, 256 codes of 512 bits, 2 eyes x 2 shifts; mid: the
# mid workload's shapes (every tile boundary of the n^2 contraction) with the chain's moduli.
CHAIN_TINY = Workload("chain_ndb512_nq512_L7_d1_256_d2_512_q4", 9, 9, 7, 7, 256, 512, 2, 2,
                      planted=(Planted(0, 17, 0, 0.1),), seed=BASE_SEED + 41)
CHAIN_MID = Workload("chain_ndb256_nq512_L7_d1_700_d2_1280_q272", 8, 9, 7, 7, 700, 1280, 17, 16,
                     seed=BASE_SEED + 42)

# The share workload with both ring degrees at 2^16 (the configuration's literal N): the same
# templates (same seed), K = 12,800 + 2^16 and 2^16 + 14,336 output rows.
PAPER_LIT = dataclasses.replace(PAPER_SHARE, name="lit_ndb65536_nq65536_L3p_d1_14336_d2_12800_q512",
                                log_n_db=16, log_n_q=16)

# Database of the batched workload: the share's shapes with five query primes, so that batch
# items can run at levels 1..5 (2..6 primes with the special prime).
PAPER_SHARE_L5 = dataclasses.replace(PAPER_SHARE, name="share_ndb16384_nq8192_L5p_d1_14336_d2_12800",
                                     n_q_primes=5, level=5)


@dataclasses.dataclass(frozen=True)
class BatchItemSpec:
    eyes: int       # query eyes of the item (columns = eyes * shifts)
    level: int      # query primes used
    row0: int       # first database code of the item's shard
    rows: int       # codes in the shard


def batched_mix(seed: int, n_items: int, d1: int, max_eyes: int, max_level: int,
                min_rows: int) -> Tuple[BatchItemSpec, ...]:
    """Uneven batch items: eyes ~ U{1..max_eyes}, level ~ U{1..max_level}, shard size
    ~ U{min_rows..d1} codes at a uniform offset."""
    g = _rng(seed, 4)
    out = []
    for _ in range(n_items):
        rows = int(g.integers(min_rows, d1 + 1))
        out.append(BatchItemSpec(eyes=int(g.integers(1, max_eyes + 1)), level=int(g.integers(1, max_level + 1)),
                                 row0=int(g.integers(0, d1 - rows + 1)), rows=rows))
    return tuple(out)


def poisson_arrivals(seed: int, n: int, rate: float, max_eyes: int) -> Tuple[np.ndarray, np.ndarray]:
    """Arrival times (seconds from 0; exponential gaps of mean 1/rate) and eyes ~ U{1..max_eyes}."""
    g = _rng(seed, 5)
    t = np.cumsum(g.exponential(1.0 / rate, n))
    return t - t[0], g.integers(1, max_eyes + 1, n)


def random_eyes(seed: int, stream: int, n_eyes: int, d2: int, p_code: float = 0.5,
                p_mask: float = 0.9) -> Tuple[np.ndarray, np.ndarray]:
    """Fresh query eyes (codes, masks), uint8 0/1 of shape (n_eyes, d2)."""
    g = _rng(seed, 100 + stream)
    return ((g.random((n_eyes, d2)) < p_code).astype(np.uint8),
            (g.random((n_eyes, d2)) < p_mask).astype(np.uint8))


# Workloads of FormatSwitch (Appendix C.1): the query arrives in a transmission ring of degree
# 2^FS_LOG_N_T[name] modulo one prime more than the CCMM level (n_q_primes = level + 1).  Tiny:
# 2^10 -> 2^7 (rho 8), two chunks per column; mid: 2^12 -> 2^9 with three chunks per column (1,100
# positions); paper: the paper's 2^16 -> 2^13 with its 12,800-bit codes at level 3; wide: 2^15 -> 2^14,
# the largest query ring (two register groups per thread in the fused transforms).
FS_TINY = Workload("fs_ndb128_nq128_nt1024_L2_d1_64_d2_200_q3", 7, 7, 3, 2, 64, 200, 3, 1,
                   planted=(Planted(0, 5, 0, 0.1),), seed=BASE_SEED + 51)
FS_FLAT = dataclasses.replace(FS_TINY, name="fs_ndb128_nq128_nt128_L1_d1_64_d2_200_q3", n_q_primes=2, level=1)
FS_MID = Workload("fs_ndb256_nq512_nt4096_L2_d1_300_d2_1100_q5", 8, 9, 3, 2, 300, 1100, 5, 1,
                  planted=(Planted(2, 100, 0, 0.1),), seed=BASE_SEED + 52)
FS_PAPER = Workload("fs_ndb16384_nq8192_nt65536_L3_d1_256_d2_12800_q2", 14, 13, 4, 3, 256, 12800, 2, 1,
                    planted=(Planted(1, 17, 0, 0.1),), seed=BASE_SEED + 53)
FS_WIDE = Workload("fs_ndb128_nq16384_nt32768_L1_d1_64_d2_300_q2", 7, 14, 2, 1, 64, 300, 2, 1,
                   planted=(Planted(0, 9, 0, 0.1),), seed=BASE_SEED + 54)
# The share workload's queries (512 columns) through FormatSwitch: its keys carry a fourth prime for
# the transmission modulus; the CCMM runs at level 3 as in the share workload.
FS_SHARE = dataclasses.replace(PAPER_SHARE, name="fs_share_ndb16384_nq8192_nt65536_L3_d1_14336_d2_12800_q512",
                               n_q_primes=4, level=3)
FS_LOG_N_T = {FS_TINY.name: 10, FS_FLAT.name: 7, FS_MID.name: 12, FS_PAPER.name: 16, FS_SHARE.name: 16,
              FS_WIDE.name: 15}

WORKLOADS: Dict[str, Workload] = {w.name: w for w in (TINY, TINY_MULTI, MID, PAPER_SHARE, PAPER_SHARE_L5, BIG_DB,
                                                      BIG_Q, PAPER_LIT, CHAIN_TINY, CHAIN_MID,
                                                      FS_TINY, FS_FLAT, FS_MID, FS_PAPER, FS_SHARE,
                                                      FS_WIDE)}


# ---------------------------------------------------------------- normalise and fold
# Inputs of the fold (Algorithm 2 after the CCMM): per score ciphertext c and slot j, the mask count
# ||m_q AND m_db||_1 (Binomial(d2, 0.81): two masks of density 0.9) and the inner product
# IP = round(score * count), with non-matching scores drawn from the normal law of Appendix C.2 (mean
# 0.008, standard deviation 0.06) clipped to [-0.233, 0.3], and one planted matching score in
# [0.35, 0.6] per group of k ciphertexts (at most one match per slot of a group: the folding
# assumption).  Slots past d1 (the database entries of the last block) hold IP 0 with count 1.

@dataclasses.dataclass(frozen=True)
class FoldWorkload:
    name: str
    log_n: int           # ring degree of the fold
    k: int               # folding factor
    rho: int             # score ciphertexts per database block (query columns)
    blocks: int          # database blocks of N/2 entries
    d2: int              # code length (scale of the mask counts)
    d1: int              # database entries (<= blocks N/2)
    seed: int

    @property
    def count(self) -> int:
        return self.blocks * self.rho


def fold_inputs(w: FoldWorkload) -> Tuple[np.ndarray, np.ndarray]:
    """(ip, counts), int32 arrays of shape (count, N/2), block-major (ciphertext b rho + c)."""
    g = _rng(w.seed, 7)
    slots = (1 << w.log_n) // 2
    counts = g.binomial(w.d2, 0.81, (w.count, slots)).astype(np.int64)
    scores = np.clip(g.normal(0.008, 0.06, (w.count, slots)), -0.233, 0.3)
    groups = -(-w.rho // w.k)
    for b in range(w.blocks):
        for r in range(groups):
            size = min(w.k, w.rho - r * w.k)
            c = b * w.rho + r * w.k + int(g.integers(0, size))
            scores[c, int(g.integers(0, slots))] = g.uniform(0.35, 0.6)
    ip = np.rint(scores * counts).astype(np.int64)
    for b in range(w.blocks):
        live = w.d1 - b * slots
        if live < slots:
            lo = max(live, 0)
            ip[b * w.rho:(b + 1) * w.rho, lo:] = 0
            counts[b * w.rho:(b + 1) * w.rho, lo:] = 1
    return ip.astype(np.int32), counts.astype(np.int32)


FOLD_TINY = FoldWorkload("fold_n128_k4_rho6_b2", 7, 4, 6, 2, 200, 120, BASE_SEED + 61)
FOLD_MID = FoldWorkload("fold_n1024_k16_rho20_b1", 10, 16, 20, 1, 1100, 512, BASE_SEED + 62)
FOLD_PAPER = FoldWorkload("fold_n16384_k16_rho16_b1", 14, 16, 16, 1, 12800, 8192, BASE_SEED + 63)
# The share workload's scores: 512 query columns against 14,336 database entries in two blocks of 8,192
# slots at the fold's ring degree 2^14 (k = 16 as in Appendix C.2).
FOLD_SHARE = FoldWorkload("fold_share_n16384_k16_rho512_b2_d1_14336", 14, 16, 512, 2, 12800, 14336, BASE_SEED + 64)
FOLD_WORKLOADS: Dict[str, FoldWorkload] = {w.name: w for w in (FOLD_TINY, FOLD_MID, FOLD_PAPER, FOLD_SHARE)}


def planted_for(w: Workload, count: int = 4) -> Tuple[Planted, ...]:
    """Planted eyes for a workload: its own list if given, else `count` random ones."""
    if w.planted:
        return w.planted
    return _planted(w.eyes, w.d1, w.n_shifts, count, w.seed)


def make_inputs(w: Workload, n_planted: int = 4) -> Dict[str, np.ndarray]:
    """All template bits of a workload: db codes/masks, eye codes/masks, shifts."""
    dbc, dbm = db_templates(w.seed, w.d1, w.d2)
    pl = planted_for(w, n_planted)
    qc, qm = query_eyes(w.seed, w.eyes, w.d2, dbc, dbm, pl)
    return dict(db_codes=dbc, db_masks=dbm, q_codes=qc, q_masks=qm,
                shifts=default_shifts(w.n_shifts), planted=pl)
