"""ctypes view of the oracle's C arithmetic (ckks_prims.c).

TEST INFRASTRUCTURE ONLY.  Thin wrappers: numpy arrays in, numpy arrays out.
Loads oracle/_prims.so, building it with gcc when it is absent.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_u64 = ctypes.c_uint64
_p = ctypes.c_void_p
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.OUT
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.or_mulmod.restype = _u64
        L.or_mulmod.argtypes = [_u64, _u64, _u64]
        L.or_powmod.restype = _u64
        L.or_powmod.argtypes = [_u64, _u64, _u64]
        L.or_invmod.restype = _u64
        L.or_invmod.argtypes = [_u64, _u64]
        L.or_find_psi.restype = _u64
        L.or_find_psi.argtypes = [_u64, _u64]
        L.or_polymul.restype = ctypes.c_int
        L.or_polymul.argtypes = [_u64, ctypes.c_size_t, _p, _p, _p]
        L.or_polymul_batch.restype = ctypes.c_int
        L.or_polymul_batch.argtypes = [ctypes.c_size_t, ctypes.c_size_t, _p, _p, _p, _p]
        L.or_polymul_schoolbook.restype = None
        L.or_polymul_schoolbook.argtypes = [_u64, ctypes.c_size_t, _p, _p, _p]
        L.or_mulmod_vec.restype = None
        L.or_mulmod_vec.argtypes = [_u64, ctypes.c_size_t, _p, _p, _p]
        L.or_mulmod_scalar.restype = None
        L.or_mulmod_scalar.argtypes = [_u64, ctypes.c_size_t, _p, _u64, _p]
        L.or_shake256.restype = None
        L.or_shake256.argtypes = [ctypes.c_char_p, ctypes.c_size_t, _p, ctypes.c_size_t]
        L.or_stream_words.restype = None
        L.or_stream_words.argtypes = [_u64, ctypes.c_uint32, _u64, _p, ctypes.c_size_t]
        L.or_sample_ternary.restype = None
        L.or_sample_ternary.argtypes = [_u64, ctypes.c_uint32, _u64, _p, ctypes.c_size_t]
        L.or_sample_cdt.restype = None
        L.or_sample_cdt.argtypes = [_u64, ctypes.c_uint32, _u64, _p, ctypes.c_size_t,
                                    ctypes.c_int64, _p, ctypes.c_size_t]
        L.or_sample_uniform.restype = None
        L.or_sample_uniform.argtypes = [_u64, ctypes.c_uint32, _u64, _p, ctypes.c_size_t,
                                        ctypes.c_size_t, _p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u64arr(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def mulmod(a, b, q):
    return int(lib().or_mulmod(int(a), int(b), int(q)))


def powmod(b, e, q):
    return int(lib().or_powmod(int(b), int(e), int(q)))


def invmod(a, q):
    return int(lib().or_invmod(int(a), int(q)))


def polymul(a, b, q):
    """Negacyclic product a*b in Z_q[X]/(X^N+1) (textbook NTT)."""
    a = _u64arr(a)
    b = _u64arr(b)
    out = np.empty_like(a)
    if lib().or_polymul(int(q), a.size, _ptr(a), _ptr(b), _ptr(out)) != 0:
        raise ValueError("q=%d has no primitive 2N-th root for N=%d" % (q, a.size))
    return out


def polymul_batch(jobs):
    """jobs: list of (a, b, q).  Returns the list of products (parallel in C)."""
    if not jobs:
        return []
    n = jobs[0][0].size
    As = [_u64arr(a) for a, _, _ in jobs]
    Bs = [_u64arr(b) for _, b, _ in jobs]
    outs = [np.empty(n, dtype=np.uint64) for _ in jobs]
    qs = np.array([int(q) for _, _, q in jobs], dtype=np.uint64)
    pa = (ctypes.c_void_p * len(jobs))(*[x.ctypes.data for x in As])
    pb = (ctypes.c_void_p * len(jobs))(*[x.ctypes.data for x in Bs])
    po = (ctypes.c_void_p * len(jobs))(*[x.ctypes.data for x in outs])
    rc = lib().or_polymul_batch(len(jobs), n, _ptr(qs), ctypes.cast(pa, _p),
                                ctypes.cast(pb, _p), ctypes.cast(po, _p))
    if rc != 0:
        raise ValueError("a modulus has no primitive 2N-th root")
    return outs


def polymul_schoolbook(a, b, q):
    a = _u64arr(a)
    b = _u64arr(b)
    out = np.empty_like(a)
    lib().or_polymul_schoolbook(int(q), a.size, _ptr(a), _ptr(b), _ptr(out))
    return out


def mulmod_vec(a, b, q):
    a = _u64arr(a)
    b = _u64arr(b)
    out = np.empty_like(a)
    lib().or_mulmod_vec(int(q), a.size, _ptr(a), _ptr(b), _ptr(out))
    return out


def mulmod_scalar(a, c, q):
    a = _u64arr(a)
    out = np.empty_like(a)
    lib().or_mulmod_scalar(int(q), a.size, _ptr(a), int(c) % int(q), _ptr(out))
    return out


def shake256(data: bytes, n: int) -> bytes:
    out = ctypes.create_string_buffer(n)
    lib().or_shake256(data, len(data), ctypes.cast(out, _p), n)
    return out.raw


def stream_words(seed, domain, index, n):
    out = np.empty(n, dtype=np.uint64)
    lib().or_stream_words(int(seed), int(domain), int(index), _ptr(out), n)
    return out


def sample_ternary(seed, domain, index, n):
    out = np.empty(n, dtype=np.int64)
    lib().or_sample_ternary(int(seed), int(domain), int(index), _ptr(out), n)
    return out


def sample_cdt(seed, domain, index, cdt, lo, n):
    cdt = _u64arr(cdt)
    out = np.empty(n, dtype=np.int64)
    lib().or_sample_cdt(int(seed), int(domain), int(index), _ptr(cdt), cdt.size, int(lo),
                        _ptr(out), n)
    return out


def sample_uniform(seed, domain, index, primes, n):
    qs = np.array([int(q) for q in primes], dtype=np.uint64)
    out = np.empty(len(primes) * n, dtype=np.uint64)
    lib().or_sample_uniform(int(seed), int(domain), int(index), _ptr(qs), qs.size, n, _ptr(out))
    return out.reshape(len(primes), n)
