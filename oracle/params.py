"""Parameters: NTT-friendly primes, ring degrees, scaling factor (oracle).

Readings taken where the paper is silent (Section 2.3, Section 6.3 and
Table 5 give only bit sizes):
  * RNS primes are ~36-bit with q = 1 (mod 2^17), so that every ring degree
    N <= 2^16 has a primitive 2N-th root of unity mod q.  They are the largest
    such primes below 2^36, in decreasing order; the first is the special
    prime p, the next ones are the query primes q_0, q_1, ...
  * The query scaling factor is Delta = 2^(floor(log2 Q) - gap) with gap = 20,
    where Q is the product of the query primes used (the level).
  * The database plaintext scale is p itself (a single special prime).
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; exact for n < 3.3e24 with the first 12 prime bases."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(count: int, bits: int = 36, two_adicity: int = 17) -> List[int]:
    """The `count` largest primes q < 2^bits with q = 1 (mod 2^two_adicity), descending."""
    step = 1 << two_adicity
    q = ((1 << bits) - 1) // step * step + 1
    if q >= (1 << bits):
        q -= step
    out = []
    while len(out) < count:
        if is_prime(q):
            out.append(q)
        q -= step
    return out


@dataclasses.dataclass(frozen=True)
class Params:
    log_n_db: int          # N_DB = 2^log_n_db, ring degree of the database layer
    log_n_q: int           # N_Q  = 2^log_n_q,  ring degree of the query layer
    q: Tuple[int, ...]     # query primes q_0..q_{L-1} carried by the database
    p: int                 # special prime (database plaintext scale, rescale divisor)
    d2: int                # code length (columns of M_DB, rows of M_Q)
    max_db_rows: int       # largest d1 the keys must cover (number of DB secrets)
    gap: int = 20          # Delta = 2^(floor(log2 Q) - gap)
    t_num: int = 3         # threshold t = t_num / t_den
    t_den: int = 8

    @property
    def n_db(self) -> int:
        return 1 << self.log_n_db

    @property
    def n_q(self) -> int:
        return 1 << self.log_n_q

    @property
    def k(self) -> int:
        """Number of query secrets: ceil(d2 / N_Q)."""
        return -(-self.d2 // self.n_q)

    @property
    def k_db(self) -> int:
        """Number of database secrets: ceil(max_db_rows / N_DB)."""
        return -(-self.max_db_rows // self.n_db)

    @property
    def K(self) -> int:
        """Contraction length of the CCMM: d2 + N_Q."""
        return self.d2 + self.n_q

    def Q(self, level: int) -> int:
        out = 1
        for qi in self.q[:level]:
            out *= qi
        return out

    def delta(self, level: int) -> int:
        Q = self.Q(level)
        return 1 << (Q.bit_length() - 1 - self.gap)


def make_params(log_n_db: int, log_n_q: int, n_q_primes: int, d2: int,
                max_db_rows: int, gap: int = 20) -> Params:
    primes = ntt_primes(n_q_primes + 1)
    return Params(log_n_db=log_n_db, log_n_q=log_n_q, q=tuple(primes[1:]), p=primes[0],
                  d2=d2, max_db_rows=max_db_rows, gap=gap)
