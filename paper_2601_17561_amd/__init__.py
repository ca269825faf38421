"""Python binding of libhfe, the MI355X encrypted-CCMM library (argument marshalling only).

Every function below has the name of the C entry point it calls (include/hfe.h) and does
nothing but convert arguments: torch tensors on the GPU become device pointers, the current
torch stream becomes the hipStream_t, handles are wrapped so that they are released with
hfe_free, and a negative status raises HfeError with hfe_last_error().  All arithmetic of
the encrypted matching runs in the HIP kernels of the library.

PyTorch provides device memory and streams: on import the binding installs torch's caching
allocator as the library's allocator (hfe_set_allocator), so the library's buffers are
stream-ordered blocks of torch's pool.

The library must have been built (paper_2601_17561_amd/build.py); importing this package
without it raises ImportError.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfe.so")

HFE_FORM_PLAIN_U64 = 1
HFE_FORM_I8_MFMA = 2
HFE_FORM_RNS_I8 = 4
HFE_FORM_P2_I8 = 8
HFE_PROBE_MFMA_I8, HFE_PROBE_MFMA_I8_ZERO, HFE_PROBE_VALU_MAD_U64 = 1, 2, 3
HFE_MAX_QPRIMES = 8
HFE_NOALLOC_SCRATCH_BYTES = 256 << 20

STATUS_NAMES = {0: "HFE_OK", -1: "HFE_EINVAL", -2: "HFE_ESHAPE", -3: "HFE_ELEVEL", -4: "HFE_ENOMEM",
                -5: "HFE_EDEVICE", -6: "HFE_EBUSY", -7: "HFE_EOVERFLOW", -8: "HFE_EINTERNAL"}

EXPORTED = ("hfe_set_allocator", "hfe_default_params", "hfe_keygen", "hfe_encode", "hfe_encrypt_db",
            "hfe_encrypt", "hfe_ccmm", "hfe_decrypt", "hfe_match", "hfe_export", "hfe_shape", "hfe_free",
            "hfe_last_error", "hfe_cdt_table", "hfe_profile", "hfe_profile_ms", "hfe_i8_variants",
            "hfe_i8_variant_name", "hfe_set_i8_variant", "hfe_ccmm_batched", "hfe_plan_create", "hfe_plan_run",
            "hfe_plan_result", "hfe_autotune", "hfe_autotune_save", "hfe_autotune_load", "hfe_server_create",
            "hfe_server_submit", "hfe_server_poll", "hfe_server_wait", "hfe_server_drain", "hfe_server_stats", "hfe_server_reset_stats",
            "hfe_db_save", "hfe_db_load", "hfe_result_create", "hfe_server_submit_encrypted", "hfe_db_bytes",
            "hfe_ccmm_product", "hfe_probe_rate", "hfe_noalloc_init", "hfe_ccmm_noalloc",
            "hfe_plan_create_for", "hfe_chain_default_params", "hfe_chain_keygen", "hfe_fs_keygen",
            "hfe_fs_transmit_count", "hfe_fs_encrypt", "hfe_format_switch", "hfe_fs_profile_ms",
            "hfe_fold_keygen", "hfe_fold_encrypt", "hfe_fold", "hfe_fold_profile_ms", "hfe_fold_decrypt")


class HfeError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class hfe_params(ctypes.Structure):
    _fields_ = [("log_n_db", ctypes.c_uint32), ("log_n_q", ctypes.c_uint32), ("n_q_primes", ctypes.c_uint32),
                ("q", ctypes.c_uint64 * HFE_MAX_QPRIMES), ("p", ctypes.c_uint64), ("gap_bits", ctypes.c_uint32),
                ("d2", ctypes.c_uint32), ("max_db_rows", ctypes.c_uint32), ("t_num", ctypes.c_uint32),
                ("t_den", ctypes.c_uint32)]

    def primes(self):
        return [int(self.q[i]) for i in range(self.n_q_primes)], int(self.p)


HFE_CHAIN_MAX_BASES = 11


class hfe_chain_params(ctypes.Structure):
    _fields_ = [("log_n_db", ctypes.c_uint32), ("log_n_q", ctypes.c_uint32), ("n_q_mods", ctypes.c_uint32),
                ("n_p_mods", ctypes.c_uint32), ("bases", ctypes.c_uint32 * HFE_CHAIN_MAX_BASES),
                ("ntt_prime", ctypes.c_uint64), ("gap_bits", ctypes.c_uint32), ("d2", ctypes.c_uint32),
                ("max_db_rows", ctypes.c_uint32), ("t_num", ctypes.c_uint32), ("t_den", ctypes.c_uint32)]

    def q_bases(self):
        return [int(self.bases[i]) for i in range(self.n_q_mods)]

    def p_bases(self):
        return [int(self.bases[self.n_q_mods + i]) for i in range(self.n_p_mods)]


class hfe_batch_item(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p), ("row0", ctypes.c_int64), ("rows", ctypes.c_int64)]


class hfe_server_report(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "steps", "max_queue")] + \
               [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "service_p50_ms", "service_p99_ms", "mean_ms",
                                               "req_per_s", "cmp_per_s", "mean_cols_per_step", "elapsed_s")] + \
               [(n, ctypes.c_int64) for n in ("retained", "max_busy_slots", "overlap_pairs")]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2601_17561_amd/build.py` "
                      "(there is no CPU fallback)")

# torch ships its own HIP and HSA runtimes under the same sonames as ROCm's.  Importing it first
# lets libhfe.so bind to those already loaded; loaded the other way round, a process would hold
# two HIP runtimes, and the library's would find no device next to torch's.
try:
    import torch as _torch_first  # noqa: F401
except ImportError:  # host-only use of the library (no device work)
    pass
_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _i64, _u32, _u64, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_size_t)
_ALLOC_FN = ctypes.CFUNCTYPE(_vp, _sz, _vp, _vp)
_DEALLOC_FN = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)

_SIGS = {
    "hfe_set_allocator": [_ALLOC_FN, _DEALLOC_FN, _vp],
    "hfe_default_params": [_u32, _u32, _u32, _u32, _u32, ctypes.POINTER(hfe_params)],
    "hfe_keygen": [ctypes.POINTER(hfe_params), _u64, ctypes.POINTER(_vp)],
    "hfe_chain_default_params": [_u32, _u32, _u32, _u32, _u32, _u32, ctypes.POINTER(hfe_chain_params)],
    "hfe_chain_keygen": [ctypes.POINTER(hfe_chain_params), _u64, ctypes.POINTER(_vp)],
    "hfe_encode": [_vp, _vp, _i64, _i32, ctypes.POINTER(_i32), _i32, _vp, _vp],
    "hfe_encrypt_db": [_vp, _vp, _i64, _u64, _u32, _vp, ctypes.POINTER(_vp)],
    "hfe_encrypt": [_vp, _vp, _i64, _u32, _u64, _vp, ctypes.POINTER(_vp)],
    "hfe_db_save": [_vp, ctypes.c_char_p, _vp],
    "hfe_db_bytes": [_vp, _u32, ctypes.POINTER(_sz)],
    "hfe_result_create": [_vp, _vp, _vp, ctypes.POINTER(_vp)],
    "hfe_server_submit_encrypted": [_vp, _vp, _vp, ctypes.POINTER(_u64)],
    "hfe_db_load": [_vp, ctypes.c_char_p, _u32, _vp, ctypes.POINTER(_vp)],
    "hfe_ccmm": [_vp, _vp, _i64, _i64, _i32, _vp, ctypes.POINTER(_vp)],
    "hfe_ccmm_product": [_vp, _vp, _i64, _i64, _i32, _vp, _vp],
    "hfe_noalloc_init": [],
    "hfe_ccmm_noalloc": [_vp, _vp, _i64, _i64, _i32, _vp, _vp],
    "hfe_decrypt": [_vp, _vp, _vp, _vp, _vp],
    "hfe_match": [_vp, _vp, _i64, ctypes.POINTER(_i32), _i32, _vp, _i64, _i32, _u32, _u32, _vp, _vp, _vp],
    "hfe_export": [_vp, _i32, _sz, _vp, _sz, ctypes.POINTER(_sz)],
    "hfe_shape": [_vp, ctypes.POINTER(_i64)],
    "hfe_cdt_table": [_vp],
    "hfe_profile": [_i32],
    "hfe_profile_ms": [_vp, _vp, _i32],
    "hfe_probe_rate": [_i32, _i64, _vp, ctypes.POINTER(ctypes.c_double)],
    "hfe_set_i8_variant": [_i32],
    "hfe_ccmm_batched": [_vp, ctypes.POINTER(hfe_batch_item), _i32, _i32, _vp, ctypes.POINTER(_vp)],
    "hfe_plan_create": [_vp, _i32, _i64, _u32, _i32, ctypes.POINTER(_vp)],
    "hfe_plan_run": [_vp, ctypes.POINTER(hfe_batch_item), _i32, _i32, _vp],
    "hfe_plan_create_for": [_vp, ctypes.POINTER(hfe_batch_item), _i32, _i32, ctypes.POINTER(_vp)],
    "hfe_plan_result": [_vp, _i32, ctypes.POINTER(_vp)],
    "hfe_autotune": [_vp, _vp, _i64, _i64, _i32, _vp, ctypes.POINTER(_i32)],
    "hfe_autotune_save": [ctypes.c_char_p],
    "hfe_autotune_load": [ctypes.c_char_p],
    "hfe_server_create": [_vp, _sz, _i64, _i32, _i32, _u32, _i32, ctypes.POINTER(_vp)],
    "hfe_server_submit": [_vp, _vp, _vp, ctypes.POINTER(_u64)],
    "hfe_server_poll": [_vp, _u64, ctypes.POINTER(_i32)],
    "hfe_server_wait": [_vp, _u64, _i64],
    "hfe_server_drain": [_vp, _i64],
    "hfe_server_stats": [_vp, ctypes.POINTER(hfe_server_report)],
    "hfe_server_reset_stats": [_vp],
    "hfe_fs_keygen": [_vp, _u32, _u32, _u64, ctypes.POINTER(_vp)],
    "hfe_fs_transmit_count": [_vp, _i64, ctypes.POINTER(_i64)],
    "hfe_fs_encrypt": [_vp, _vp, _i64, _u64, _vp, _vp],
    "hfe_format_switch": [_vp, _vp, _i64, _vp, ctypes.POINTER(_vp)],
    "hfe_fs_profile_ms": [_vp, _vp, _i32],
    "hfe_fold_keygen": [_u32, _u32, _u32, _u64, ctypes.POINTER(_vp)],
    "hfe_fold_encrypt": [_vp, _vp, _i64, _u64, _vp, ctypes.POINTER(_vp)],
    "hfe_fold": [_vp, _vp, _vp, _i64, _vp, ctypes.POINTER(_vp)],
    "hfe_fold_profile_ms": [_vp, _vp, _i32],
    "hfe_fold_decrypt": [_vp, _vp, _vp, _vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _i32
_lib.hfe_free.argtypes = [_vp]
_lib.hfe_free.restype = None
_lib.hfe_i8_variants.argtypes = []
_lib.hfe_i8_variants.restype = _i32
_lib.hfe_i8_variant_name.argtypes = [_i32]
_lib.hfe_i8_variant_name.restype = ctypes.c_char_p
_lib.hfe_last_error.argtypes = []
_lib.hfe_last_error.restype = ctypes.c_char_p


def hfe_last_error() -> str:
    return _lib.hfe_last_error().decode()


def _check(status: int, fn: str) -> None:
    if status != 0:
        raise HfeError(status, fn, hfe_last_error())


# ------------------------------------------------------------------ torch plumbing

def _torch():
    import torch
    return torch


def _stream(stream) -> int:
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, dtype) -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


_allocator_refs = []


def hfe_set_allocator(alloc=None, dealloc=None, ctx=None) -> None:
    """Install Python callables alloc(bytes, stream) -> int and dealloc(ptr, stream)."""
    if alloc is None:
        _check(_lib.hfe_set_allocator(_ALLOC_FN(), _DEALLOC_FN(), None), "hfe_set_allocator")
        _allocator_refs.clear()
        return

    def _a(nbytes, stream, _ctx):
        try:
            return alloc(int(nbytes), int(stream or 0))
        except Exception:  # allocation failure is reported as NULL -> HFE_ENOMEM
            return None

    def _d(ptr, stream, _ctx):
        try:
            dealloc(int(ptr), int(stream or 0))
        except Exception:
            pass

    a, d = _ALLOC_FN(_a), _DEALLOC_FN(_d)
    _allocator_refs[:] = [a, d]
    _check(_lib.hfe_set_allocator(a, d, None), "hfe_set_allocator")


def use_torch_allocator() -> None:
    """Route the library's device memory through torch's caching allocator."""
    torch = _torch()

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def dealloc(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    hfe_set_allocator(alloc, dealloc)


# ------------------------------------------------------------------ handles

class Handle:
    """Owner of a library handle; released with hfe_free when collected or on free()."""

    def __init__(self, ptr: int, parents=()):
        self.ptr = ptr
        self._parents = tuple(parents)

    def free(self) -> None:
        if self.ptr:
            _lib.hfe_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def as_parameter(self):
        return self.ptr


def hfe_shape(h: Handle):
    dims = (_i64 * 4)()
    _check(_lib.hfe_shape(h.ptr, dims), "hfe_shape")
    return tuple(int(x) for x in dims)


def hfe_free(h: Handle) -> None:
    h.free()


# ------------------------------------------------------------------ entry points

def hfe_default_params(log_n_db: int, log_n_q: int, n_q_primes: int, d2: int, max_db_rows: int) -> hfe_params:
    P = hfe_params()
    _check(_lib.hfe_default_params(log_n_db, log_n_q, n_q_primes, d2, max_db_rows, ctypes.byref(P)),
           "hfe_default_params")
    return P


def hfe_keygen(params: hfe_params, seed: int) -> Handle:
    out = _vp()
    _check(_lib.hfe_keygen(ctypes.byref(params), seed, ctypes.byref(out)), "hfe_keygen")
    return Handle(out.value)


def hfe_chain_default_params(log_n_db: int, log_n_q: int, n_q_mods: int, n_p_mods: int, d2: int,
                             max_db_rows: int) -> hfe_chain_params:
    C = hfe_chain_params()
    _check(_lib.hfe_chain_default_params(log_n_db, log_n_q, n_q_mods, n_p_mods, d2, max_db_rows, ctypes.byref(C)),
           "hfe_chain_default_params")
    return C


def hfe_chain_keygen(params: hfe_chain_params, seed: int) -> Handle:
    out = _vp()
    _check(_lib.hfe_chain_keygen(ctypes.byref(params), seed, ctypes.byref(out)), "hfe_chain_keygen")
    return Handle(out.value)


def hfe_fs_keygen(keys: Handle, level: int, log_n_t: int, seed: int) -> Handle:
    """FormatSwitch keys (Appendix C.1) for queries of level `level` from ring degree 2^log_n_t."""
    out = _vp()
    _check(_lib.hfe_fs_keygen(keys.ptr, level, log_n_t, seed, ctypes.byref(out)), "hfe_fs_keygen")
    return Handle(out.value, (keys,))


def hfe_fs_transmit_count(fk: Handle, d3: int) -> int:
    n = _i64()
    _check(_lib.hfe_fs_transmit_count(fk.ptr, d3, ctypes.byref(n)), "hfe_fs_transmit_count")
    return int(n.value)


def hfe_fs_encrypt(fk: Handle, m_q, seed: int, T=None, stream=None):
    """Transmission ciphertexts of M_Q (d3 x d2 int8 GPU tensor): uint64 residues as an int64 GPU tensor,
    layout [prime i <= level][d3 k][a | b][N_T] (flat)."""
    torch = _torch()
    d3 = m_q.shape[0]
    if T is None:
        T = torch.empty(hfe_fs_transmit_count(fk, d3), dtype=torch.int64, device=m_q.device)
    _check(_lib.hfe_fs_encrypt(fk.ptr, _dev_ptr(m_q, torch.int8), d3, seed, _dev_ptr(T, torch.int64),
                               _stream(stream)), "hfe_fs_encrypt")
    return T


def hfe_format_switch(fk: Handle, T, d3: int, stream=None) -> Handle:
    """Query ciphertext (for hfe_ccmm) from the transmission ciphertexts T of d3 query columns."""
    torch = _torch()
    out = _vp()
    _check(_lib.hfe_format_switch(fk.ptr, _dev_ptr(T, torch.int64), d3, _stream(stream), ctypes.byref(out)),
           "hfe_format_switch")
    return Handle(out.value, (fk,))


def hfe_fs_profile_ms(q: Handle, n: int = 4):
    ms = (ctypes.c_float * n)()
    _check(_lib.hfe_fs_profile_ms(q.ptr, ms, n), "hfe_fs_profile_ms")
    return [float(x) for x in ms]


def hfe_fold_keygen(log_n: int, k: int, rho: int, seed: int) -> Handle:
    """Keys of the fold (Algorithm 2): secret, relinearisation and rotation keys at ring degree 2^log_n."""
    out = _vp()
    _check(_lib.hfe_fold_keygen(log_n, k, rho, seed, ctypes.byref(out)), "hfe_fold_keygen")
    return Handle(out.value)


def hfe_fold_encrypt(fk: Handle, ip, seed: int, stream=None) -> Handle:
    """Encryption of inner products ip (count x N/2 int32 GPU tensor) at level 4."""
    torch = _torch()
    out = _vp()
    _check(_lib.hfe_fold_encrypt(fk.ptr, _dev_ptr(ip, torch.int32), ip.shape[0], seed, _stream(stream),
                                 ctypes.byref(out)), "hfe_fold_encrypt")
    return Handle(out.value, (fk,))


def hfe_fold(fk: Handle, ct: Handle, counts, rho: int, stream=None) -> Handle:
    """The fold of ct in blocks of rho with the mask counts (count x N/2 int32 GPU tensor)."""
    torch = _torch()
    out = _vp()
    _check(_lib.hfe_fold(fk.ptr, ct.ptr, _dev_ptr(counts, torch.int32), rho, _stream(stream), ctypes.byref(out)),
           "hfe_fold")
    return Handle(out.value, (fk,))


def hfe_fold_profile_ms(ct: Handle, n: int = 4):
    ms = (ctypes.c_float * n)()
    _check(_lib.hfe_fold_profile_ms(ct.ptr, ms, n), "hfe_fold_profile_ms")
    return [float(x) for x in ms]


def hfe_fold_decrypt(fk: Handle, ct: Handle, values=None, stream=None):
    """Slot values of folded ciphertexts: a count x N/2 float64 GPU tensor."""
    torch = _torch()
    level, count, n, _ = hfe_shape(ct)
    if values is None:
        values = torch.empty((count, n // 2), dtype=torch.float64, device="cuda")
    _check(_lib.hfe_fold_decrypt(fk.ptr, ct.ptr, _dev_ptr(values, torch.float64), _stream(stream)),
           "hfe_fold_decrypt")
    return values


def hfe_encode(codes, masks, shifts: Sequence[int], out=None, stream=None):
    """codes, masks: uint8 (n x d2) GPU tensors; returns int8 ((n * len(shifts)) x d2)."""
    torch = _torch()
    n, d2 = codes.shape
    sh = (_i32 * len(shifts))(*[int(s) for s in shifts])
    if out is None:
        out = torch.empty((n * len(shifts), d2), dtype=torch.int8, device=codes.device)
    _check(_lib.hfe_encode(_dev_ptr(codes, torch.uint8), _dev_ptr(masks, torch.uint8), n, d2, sh, len(shifts),
                           _dev_ptr(out, torch.int8), _stream(stream)), "hfe_encode")
    return out


def hfe_encrypt_db(keys: Handle, m_db, seed: int, forms: int = HFE_FORM_PLAIN_U64 | HFE_FORM_I8_MFMA,
                   stream=None) -> Handle:
    torch = _torch()
    d1 = m_db.shape[0]
    out = _vp()
    _check(_lib.hfe_encrypt_db(keys.ptr, _dev_ptr(m_db, torch.int8), d1, seed, forms, _stream(stream),
                               ctypes.byref(out)), "hfe_encrypt_db")
    return Handle(out.value, (keys,))


def hfe_db_save(db: Handle, path, stream=None) -> None:
    """Write the encrypted database (every prepared form) to `path`; returns when the file is complete."""
    _check(_lib.hfe_db_save(db.ptr, os.fsencode(path), _stream(stream)), "hfe_db_save")


def hfe_db_bytes(db: Handle, form: int = 0) -> int:
    """Device bytes the database holds for one form (0: all its forms)."""
    out = _sz()
    _check(_lib.hfe_db_bytes(db.ptr, form, ctypes.byref(out)), "hfe_db_bytes")
    return int(out.value)


def hfe_db_load(keys: Handle, path, forms: int = 0, stream=None) -> Handle:
    """Read a database written by hfe_db_save under the same keys back onto the device; forms: the
    subset of the stored forms to load (0: all)."""
    out = _vp()
    _check(_lib.hfe_db_load(keys.ptr, os.fsencode(path), forms, _stream(stream), ctypes.byref(out)), "hfe_db_load")
    return Handle(out.value, (keys,))


def hfe_encrypt(keys: Handle, m_q, level: int, seed: int, stream=None) -> Handle:
    torch = _torch()
    out = _vp()
    _check(_lib.hfe_encrypt(keys.ptr, _dev_ptr(m_q, torch.int8), m_q.shape[0], level, seed, _stream(stream),
                            ctypes.byref(out)), "hfe_encrypt")
    return Handle(out.value, (keys,))


def hfe_ccmm(db: Handle, q: Handle, row0: int, rows: int, form: int, stream=None) -> Handle:
    out = _vp()
    _check(_lib.hfe_ccmm(db.ptr, q.ptr, row0, rows, form, _stream(stream), ctypes.byref(out)), "hfe_ccmm")
    return Handle(out.value, (db, q))


def hfe_ccmm_product(db: Handle, q: Handle, row0: int, rows: int, form: int, C=None, stream=None):
    """The exact product before the rescale: uint64 GPU tensor ((level + 1) x d3 x (N_DB + rows)),
    viewed as int64 (residues < 2^36).  For the n^2 chain pass C of (level + n_p_mods) rows."""
    torch = _torch()
    level, d3, _, _ = hfe_shape(q)
    n_db = hfe_shape(db)[2] - hfe_shape(db)[1]
    if C is None:
        C = torch.empty((level + 1, d3, n_db + rows), dtype=torch.int64,
                        device=torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.hfe_ccmm_product(db.ptr, q.ptr, row0, rows, form, _stream(stream), _dev_ptr(C, torch.int64)),
           "hfe_ccmm_product")
    return C


def hfe_noalloc_init() -> None:
    _check(_lib.hfe_noalloc_init(), "hfe_noalloc_init")


def hfe_ccmm_noalloc(db: Handle, q: Handle, row0: int, rows: int, form: int, out, stream=None):
    """The allocation-free CCMM: the rescaled residues into `out`, a caller-allocated int64 GPU
    tensor of level x d3 x (N_DB + rows) (uint64 residues < 2^36); returns out."""
    torch = _torch()
    level, d3, _, _ = hfe_shape(q)
    n_db = hfe_shape(db)[2] - hfe_shape(db)[1]
    if out.numel() < level * d3 * (n_db + rows):
        raise ValueError(f"out holds {out.numel()} residues, the call writes {level * d3 * (n_db + rows)}")
    _check(_lib.hfe_ccmm_noalloc(db.ptr, q.ptr, row0, rows, form, _dev_ptr(out, torch.int64), _stream(stream)),
           "hfe_ccmm_noalloc")
    return out


def hfe_decrypt(keys: Handle, r: Handle, v=None, ip=None, stream=None):
    """Returns (v float64 or None, ip int32), both (d3 x rows) GPU tensors."""
    torch = _torch()
    _, d3, rows, _ = hfe_shape(r)
    dev = torch.device("cuda", torch.cuda.current_device())
    if ip is None:
        ip = torch.empty((d3, rows), dtype=torch.int32, device=dev)
    vp = None if v is False else (v if v is not None else torch.empty((d3, rows), dtype=torch.float64, device=dev))
    _check(_lib.hfe_decrypt(keys.ptr, r.ptr, _dev_ptr(vp, torch.float64) if vp is not None else None,
                            _dev_ptr(ip, torch.int32), _stream(stream)), "hfe_decrypt")
    return vp, ip


def hfe_match(ip, q_masks, shifts: Sequence[int], db_masks, t_num: int = 3, t_den: int = 8,
              decision=None, eye_match=None, want_decision: bool = True, stream=None):
    """Returns (decision uint8 (d3 x rows) or None, eye_match uint8 (n_eyes,))."""
    torch = _torch()
    n_eyes, d2 = q_masks.shape
    rows = db_masks.shape[0]
    sh = (_i32 * len(shifts))(*[int(s) for s in shifts])
    if want_decision and decision is None:
        decision = torch.empty((n_eyes * len(shifts), rows), dtype=torch.uint8, device=ip.device)
    if eye_match is None:
        eye_match = torch.empty((n_eyes,), dtype=torch.uint8, device=ip.device)
    _check(_lib.hfe_match(_dev_ptr(ip, torch.int32), _dev_ptr(q_masks, torch.uint8), n_eyes, sh, len(shifts),
                          _dev_ptr(db_masks, torch.uint8), rows, d2, t_num, t_den,
                          _dev_ptr(decision, torch.uint8) if decision is not None else None,
                          _dev_ptr(eye_match, torch.uint8), _stream(stream)), "hfe_match")
    return decision, eye_match


def hfe_export(h: Handle, which: int = 0, offset: int = 0, n: Optional[int] = None) -> np.ndarray:
    """Elements [offset, offset + n) of the handle's canonical residue order (all by default)."""
    total = _sz()
    _check(_lib.hfe_export(h.ptr, which, 0, None, 0, ctypes.byref(total)), "hfe_export")
    n = total.value - offset if n is None else n
    out = np.empty(n, dtype=np.uint64)
    _check(_lib.hfe_export(h.ptr, which, offset, out.ctypes.data, n, None), "hfe_export")
    return out


def hfe_profile(enable: bool) -> None:
    _check(_lib.hfe_profile(1 if enable else 0), "hfe_profile")


def hfe_profile_ms(r: Handle, n: int = 3) -> list:
    """Stage durations (ms) of a profiled hfe_ccmm: [lift + split, contraction, rescale][:n]."""
    out = (ctypes.c_float * 3)()
    _check(_lib.hfe_profile_ms(r.ptr, out, n), "hfe_profile_ms")
    return [float(out[i]) for i in range(n)]


def hfe_probe_rate(which: int, iters: int, stream=None) -> float:
    """Measured instruction rate of a probe (int8 ops/s for the MFMA probes, multiply-adds/s for
    the VALU probe); synchronises the stream."""
    out = ctypes.c_double()
    _check(_lib.hfe_probe_rate(which, iters, _stream(stream), ctypes.byref(out)), "hfe_probe_rate")
    return float(out.value)


def hfe_i8_variants() -> int:
    return int(_lib.hfe_i8_variants())


def hfe_i8_variant_name(v: int) -> Optional[str]:
    name = _lib.hfe_i8_variant_name(v)
    return name.decode() if name is not None else None


def hfe_set_i8_variant(v: int) -> None:
    _check(_lib.hfe_set_i8_variant(v), "hfe_set_i8_variant")


class View(Handle):
    """A result owned by a plan (valid until the plan's next run); never released here."""

    def free(self) -> None:
        self.ptr = None


def _items(items):
    arr = (hfe_batch_item * len(items))()
    for i, (q, row0, rows) in enumerate(items):
        arr[i].q = q.ptr
        arr[i].row0 = row0
        arr[i].rows = rows
    return arr


def hfe_ccmm_batched(db: Handle, items, form: int, stream=None):
    """items: sequence of (query Handle, row0, rows); returns one result Handle per item."""
    arr = _items(items)
    outs = (_vp * len(items))()
    _check(_lib.hfe_ccmm_batched(db.ptr, arr, len(items), form, _stream(stream), outs), "hfe_ccmm_batched")
    return [Handle(outs[i], (db, items[i][0])) for i in range(len(items))]


def hfe_plan_create(db: Handle, max_items: int, max_cols: int, max_level: int,
                    form: int = HFE_FORM_I8_MFMA) -> Handle:
    out = _vp()
    _check(_lib.hfe_plan_create(db.ptr, max_items, max_cols, max_level, form, ctypes.byref(out)), "hfe_plan_create")
    return Handle(out.value, (db,))


def hfe_plan_create_for(db: Handle, items, form: int = HFE_FORM_I8_MFMA) -> Handle:
    """A plan whose workspace is sized for this batch of (query Handle, row0, rows) items."""
    arr = _items(items)
    out = _vp()
    _check(_lib.hfe_plan_create_for(db.ptr, arr, len(items), form, ctypes.byref(out)), "hfe_plan_create_for")
    return Handle(out.value, (db,))


def hfe_plan_run(plan: Handle, items, use_graph: bool = True, stream=None) -> None:
    arr = _items(items)
    plan._run_items = list(items)  # keep the queries alive while the run may still read them
    _check(_lib.hfe_plan_run(plan.ptr, arr, len(items), 1 if use_graph else 0, _stream(stream)), "hfe_plan_run")


def hfe_plan_result(plan: Handle, i: int) -> View:
    out = _vp()
    _check(_lib.hfe_plan_result(plan.ptr, i, ctypes.byref(out)), "hfe_plan_result")
    return View(out.value, (plan,))


def hfe_autotune(db: Handle, q: Handle, row0: int, rows: int, reps: int = 2, stream=None) -> int:
    best = _i32()
    _check(_lib.hfe_autotune(db.ptr, q.ptr, row0, rows, reps, _stream(stream), ctypes.byref(best)), "hfe_autotune")
    return int(best.value)


def hfe_autotune_save(path: str) -> None:
    _check(_lib.hfe_autotune_save(path.encode()), "hfe_autotune_save")


def hfe_autotune_load(path: str) -> None:
    _check(_lib.hfe_autotune_load(path.encode()), "hfe_autotune_load")


class Server(Handle):
    """A serving loop; keeps each in-flight request's query and output alive until it completes."""

    def __init__(self, ptr, parents=()):
        super().__init__(ptr, parents)
        self._live = {}

    def _keep(self, ticket: int, refs) -> None:
        # the server forgets finished tickets beyond its retention window; drop the references of
        # every ticket it no longer runs, so that a long-lived server does not grow this table
        self._live[ticket] = refs
        if len(self._live) > 4096:
            st = _i32()
            for tk in list(self._live):
                if _lib.hfe_server_poll(self.ptr, tk, ctypes.byref(st)) != 0 or st.value == 2 or st.value < 0:
                    del self._live[tk]


def hfe_server_create(db: Handle, mem_budget: int, max_cols_per_step: int, max_items_per_step: int = 64,
                      n_slots: int = 2, max_level: int = 1, form: int = HFE_FORM_I8_MFMA) -> Server:
    out = _vp()
    _check(_lib.hfe_server_create(db.ptr, mem_budget, max_cols_per_step, max_items_per_step, n_slots, max_level,
                                  form, ctypes.byref(out)), "hfe_server_create")
    return Server(out.value, (db,))


def hfe_server_submit(srv: Server, q: Handle, ip_out) -> int:
    """ip_out: int32 GPU tensor (d3 x d1) receiving the request's decrypted inner products."""
    torch = _torch()
    t = _u64()
    _check(_lib.hfe_server_submit(srv.ptr, q.ptr, _dev_ptr(ip_out, torch.int32), ctypes.byref(t)), "hfe_server_submit")
    srv._keep(int(t.value), (q, ip_out))
    return int(t.value)


def hfe_result_create(db: Handle, q: Handle, stream=None) -> Handle:
    """An empty encrypted-result handle shaped for query q against every database code."""
    out = _vp()
    _check(_lib.hfe_result_create(db.ptr, q.ptr, _stream(stream), ctypes.byref(out)), "hfe_result_create")
    return Handle(out.value, (db, q))


def hfe_server_submit_encrypted(srv: Server, q: Handle, result: Handle) -> int:
    """result: a handle from hfe_result_create for q; receives the request's encrypted result."""
    t = _u64()
    _check(_lib.hfe_server_submit_encrypted(srv.ptr, q.ptr, result.ptr, ctypes.byref(t)),
           "hfe_server_submit_encrypted")
    srv._keep(int(t.value), (q, result))
    return int(t.value)


def hfe_server_poll(srv: Server, ticket: int) -> int:
    st = _i32()
    _check(_lib.hfe_server_poll(srv.ptr, ticket, ctypes.byref(st)), "hfe_server_poll")
    if st.value == 2 or st.value < 0:
        srv._live.pop(ticket, None)
    return int(st.value)


def hfe_server_wait(srv: Server, ticket: int, timeout_ms: int = -1) -> None:
    try:
        _check(_lib.hfe_server_wait(srv.ptr, ticket, timeout_ms), "hfe_server_wait")
    finally:
        st = _i32()
        if _lib.hfe_server_poll(srv.ptr, ticket, ctypes.byref(st)) == 0 and (st.value == 2 or st.value < 0):
            srv._live.pop(ticket, None)


def hfe_server_drain(srv: Server, timeout_ms: int = -1) -> None:
    """Block until nothing is queued or running on the server."""
    _check(_lib.hfe_server_drain(srv.ptr, timeout_ms), "hfe_server_drain")
    srv._live.clear()


def hfe_server_stats(srv: Server) -> dict:
    r = hfe_server_report()
    _check(_lib.hfe_server_stats(srv.ptr, ctypes.byref(r)), "hfe_server_stats")
    return {name: getattr(r, name) for name, _ in hfe_server_report._fields_}


def hfe_server_reset_stats(srv: Server) -> None:
    _check(_lib.hfe_server_reset_stats(srv.ptr), "hfe_server_reset_stats")


def hfe_cdt_table() -> list:
    out = (_u64 * 19)()
    _check(_lib.hfe_cdt_table(out), "hfe_cdt_table")
    return [int(x) for x in out]


try:  # torch's caching allocator serves the library's device memory when a GPU is present
    if _torch().cuda.is_available():
        use_torch_allocator()
except Exception:  # pragma: no cover - torch without GPU support
    pass
