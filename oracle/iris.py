"""Masked ternary encoding, query shifts and the plaintext matching truth (oracle).

Section 2.1.3: for a template (c, m) the masked vector is c' = m - 2 (c AND m)
in {-1, 0, 1}, and for two templates
    2 <c1 XOR c2, m1 AND m2> = |m1 AND m2|_1 - <c1', c2'>,
so the inner product the CCMM computes is
    IP = popcount(m1 AND m2) - 2 popcount((c1 XOR c2) AND m1 AND m2),
computed here by brute-force popcount on packed words.  The decision of
equation (2) is score = IP / popcount(m1 AND m2) > 1 - 2t, taken in exact
integers as IP * t_den > (t_den - 2 t_num) * popcount(m1 AND m2) (no match when
the masks do not overlap).  Section 2.1.2: a query eye is rotated (code and
mask together) by each shift r; here rotation by r is numpy.roll(x, r).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def ternary(codes: np.ndarray, masks: np.ndarray) -> np.ndarray:
    """c' = m - 2 (c AND m), int8."""
    c = codes.astype(np.int16)
    m = masks.astype(np.int16)
    return (m - 2 * (c & m)).astype(np.int8)


def shifted_queries(codes: np.ndarray, masks: np.ndarray, shifts: np.ndarray
                    ) -> Tuple[np.ndarray, np.ndarray]:
    """Query columns in eye-major order: column e * len(shifts) + s is eye e rolled by shifts[s]."""
    qc = np.stack([np.roll(codes[e], int(r)) for e in range(codes.shape[0]) for r in shifts])
    qm = np.stack([np.roll(masks[e], int(r)) for e in range(masks.shape[0]) for r in shifts])
    return qc, qm


def _pack(bits: np.ndarray) -> np.ndarray:
    """Rows of 0/1 bits packed into uint64 words (little-endian bit order, zero padded)."""
    n, d = bits.shape
    w = -(-d // 64)
    padded = np.zeros((n, w * 64), dtype=np.uint8)
    padded[:, :d] = bits
    return np.packbits(padded.reshape(n, w, 64)[:, :, ::-1], axis=-1).view(">u8").astype(np.uint64).reshape(n, w)


def truth(q_codes: np.ndarray, q_masks: np.ndarray, db_codes: np.ndarray, db_masks: np.ndarray
          ) -> Tuple[np.ndarray, np.ndarray]:
    """(IP*, overlap): both (n_q x n_db) int64, by popcount of packed words."""
    qc, qm = _pack(q_codes), _pack(q_masks)
    dc, dm = _pack(db_codes), _pack(db_masks)
    ip = np.empty((qc.shape[0], dc.shape[0]), dtype=np.int64)
    ov = np.empty_like(ip)
    for c in range(qc.shape[0]):
        both = qm[c][None, :] & dm
        diff = (qc[c][None, :] ^ dc) & both
        nb = np.bitwise_count(both).sum(axis=1).astype(np.int64)
        nd = np.bitwise_count(diff).sum(axis=1).astype(np.int64)
        ov[c] = nb
        ip[c] = nb - 2 * nd
    return ip, ov


def decide(ip: np.ndarray, overlap: np.ndarray, t_num: int = 3, t_den: int = 8) -> np.ndarray:
    """Match decision per pair: overlap > 0 and IP * t_den > (t_den - 2 t_num) * overlap."""
    return (overlap > 0) & (ip * t_den > (t_den - 2 * t_num) * overlap)


def match_per_eye(decisions: np.ndarray, n_shifts: int) -> np.ndarray:
    """OR over each eye's shift columns and over all database rows."""
    d3, _ = decisions.shape
    return decisions.reshape(d3 // n_shifts, n_shifts * decisions.shape[1]).any(axis=1)
