"""Oracle results for the test workloads, computed once per test session.

Each case runs the CPU oracle end to end on a seeded synthetic workload:
keys, database and query encryption, CCMM, decryption, plus the popcount truth.
GPU parity tests compare the HIP library against these values.
"""
import dataclasses
import functools
from typing import Dict

import numpy as np

import hfe_synth as S
from oracle import chain as OCH
from oracle import ckks as OC
from oracle import iris as OI
from oracle import params as OP

KEY_SEED = 101
DB_SEED = 202
Q_SEED = 303


@dataclasses.dataclass
class Case:
    w: S.Workload
    P: OP.Params
    keys: OC.Keys
    inputs: Dict
    m_db: np.ndarray
    q_codes: np.ndarray       # shifted query columns (d3 x d2)
    q_masks: np.ndarray
    m_q: np.ndarray
    D: Dict[int, np.ndarray]
    XT: Dict[int, np.ndarray]
    row0: int
    rows: int
    out: Dict[int, np.ndarray]
    v: list
    ip: np.ndarray
    ip_true: np.ndarray
    overlap: np.ndarray


def params_for(w: S.Workload) -> OP.Params:
    return OP.make_params(w.log_n_db, w.log_n_q, w.n_q_primes, w.d2, w.d1)


@functools.lru_cache(maxsize=None)
def case(name: str, row0: int = 0, rows: int = -1) -> Case:
    w = S.WORKLOADS[name]
    P = params_for(w)
    inp = S.make_inputs(w)
    keys = OC.keygen(P, KEY_SEED)
    m_db = OI.ternary(inp["db_codes"], inp["db_masks"])
    qc, qm = OI.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    m_q = OI.ternary(qc, qm)
    D = OC.encrypt_db(keys, m_db, DB_SEED)
    XT = OC.encrypt_query(keys, m_q, w.level, Q_SEED)
    rows = w.d1 - row0 if rows < 0 else rows
    out = OC.ccmm(P, D, XT, w.level, row0, rows)
    v, ip = OC.decrypt(keys, out, w.level, row0, rows)
    ip_true, ov = OI.truth(qc, qm, inp["db_codes"][row0:row0 + rows], inp["db_masks"][row0:row0 + rows])
    return Case(w, P, keys, inp, m_db, qc, qm, m_q, D, XT, row0, rows, out, v, ip, ip_true, ov)


CHAIN_P_MODS = 3   # moduli of the chain's special part P in the test workloads


@dataclasses.dataclass
class ChainCase:
    w: S.Workload
    C: OCH.ChainParams
    keys: OC.Keys
    inputs: Dict
    m_db: np.ndarray
    q_codes: np.ndarray
    q_masks: np.ndarray
    m_q: np.ndarray
    D: Dict[int, np.ndarray]
    XT: Dict[int, np.ndarray]
    level: int
    out: Dict[int, np.ndarray]
    v: list
    ip: np.ndarray
    ip_true: np.ndarray
    overlap: np.ndarray


@functools.lru_cache(maxsize=None)
def chain_case(name: str, level: int = -1) -> ChainCase:
    """The oracle end to end over the n^2 modulus chain (query moduli: the workload's n_q_primes;
    special part: CHAIN_P_MODS), at `level` query moduli (default: all)."""
    w = S.WORKLOADS[name]
    C = OCH.make_chain_params(w.log_n_db, w.log_n_q, w.n_q_primes, CHAIN_P_MODS, w.d2, w.d1)
    level = w.n_q_primes if level < 0 else level
    inp = S.make_inputs(w)
    keys = OCH.chain_keygen(C, KEY_SEED)
    m_db = OI.ternary(inp["db_codes"], inp["db_masks"])
    qc, qm = OI.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    m_q = OI.ternary(qc, qm)
    D = OCH.encrypt_db(C, keys, m_db, DB_SEED)
    XT = OCH.encrypt_query(C, keys, m_q, level, Q_SEED)
    out = OCH.ccmm(C, D, XT, level, 0, w.d1)
    v, ip = OCH.decrypt(C, keys, out, level, 0, w.d1)
    ip_true, ov = OI.truth(qc, qm, inp["db_codes"], inp["db_masks"])
    return ChainCase(w, C, keys, inp, m_db, qc, qm, m_q, D, XT, level, out, v, ip, ip_true, ov)


TX_SEED = 404      # seed of the transmission encryption in the FormatSwitch cases


@dataclasses.dataclass
class FsCase:
    w: S.Workload
    log_n_t: int
    P: OP.Params
    F: object                 # oracle.formatswitch.FSKeys
    inputs: Dict
    q_codes: np.ndarray
    q_masks: np.ndarray
    m_q: np.ndarray
    T: np.ndarray             # [prime i <= level][d3 k][a | b][N_T], the library's layout
    XT: np.ndarray            # [prime i < level][d3][d2 + N_Q]
    ip_true: np.ndarray       # popcount truth of every query column against every database code


@functools.lru_cache(maxsize=None)
def fs_case(name: str) -> FsCase:
    """FormatSwitch (Appendix C.1) of a workload's queries: keys from KEY_SEED (the CCMM keys and the
    switch's own), transmission ciphertexts from TX_SEED, the switched query, the popcount truth."""
    from oracle import formatswitch as FS
    w = S.WORKLOADS[name]
    log_n_t = S.FS_LOG_N_T[name]
    P = params_for(w)
    F = FS.fs_keygen(P, w.level, log_n_t, KEY_SEED)
    inp = S.make_inputs(w)
    qc, qm = OI.shifted_queries(inp["q_codes"], inp["q_masks"], inp["shifts"])
    m_q = OI.ternary(qc, qm)
    ct = FS.encrypt_transmit(F, m_q, TX_SEED)
    XTd = FS.format_switch(F, ct, m_q.shape[0])
    T = np.stack([ct[q] for q in F.primes_in()])
    XT = np.stack([XTd[i] for i in range(w.level)])
    ip_true, _ = OI.truth(qc, qm, inp["db_codes"], inp["db_masks"])
    return FsCase(w, log_n_t, P, F, inp, qc, qm, m_q, T, XT, ip_true)


FOLD_SEED = 707    # stream seed of the fold's input encryptions


@dataclasses.dataclass
class FoldCase:
    w: S.FoldWorkload
    P: object
    keys: object
    ip: np.ndarray
    counts: np.ndarray
    cts: list
    out: list


def fold_layout(P, cts) -> np.ndarray:
    """Oracle ciphertexts -> the library's export layout [count][b | a][q_0 .. q_level][N]."""
    lvl = cts[0][0]
    arr = np.zeros((len(cts), 2, lvl + 1, P.n), dtype=np.int64)
    for c, (l, b, a) in enumerate(cts):
        for z in range(lvl + 1):
            arr[c, 0, z] = b[P.q[z]]
            arr[c, 1, z] = a[P.q[z]]
    return arr


@functools.lru_cache(maxsize=None)
def fold_case(name: str) -> FoldCase:
    from oracle import fold as OF
    w = S.FOLD_WORKLOADS[name]
    P = OF.fold_params(w.log_n, w.k)
    keys = OF.fold_keygen(P, KEY_SEED, OF.rot_amounts(w.k, w.rho))
    ip, counts = S.fold_inputs(w)
    cts = [OF.encrypt(keys, ip[c], FOLD_SEED, c) for c in range(w.count)]
    out = OF.fold(keys, cts, counts, w.rho)
    return FoldCase(w, P, keys, ip, counts, cts, out)
