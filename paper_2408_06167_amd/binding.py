"""ctypes binding of libblindmatch.so: the C entry points under the same names.

Argument marshalling only (numpy arrays in and out, handles as opaque
pointers, non-zero status raised as BMError); every step of the computation
runs inside the library.  Importing this module does not need a GPU, but the
library must have been built (`paper_2408_06167_amd.build.build()`): there is
no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblindmatch.so")

BM_OK, BM_EINVAL, BM_EDIM, BM_ELEVEL, BM_ESCALE, BM_ENOKEY = 0, -1, -2, -3, -4, -5
BM_ENOMEM, BM_EBUDGET, BM_EDEVICE, BM_EBUSY = -6, -7, -8, -9
BM_S1, BM_S2 = 1, 2
BM_LEVEL_MIN = 0x100
BM_COMPRESS = 0x200
BM_HOIST = 0x400
BM_RING_STD, BM_RING_CI = 0, 1


class BMError(RuntimeError):
    def __init__(self, code, fn, detail):
        super().__init__("%s failed: %s (%d) %s" % (fn, _strerror(code), code, detail))
        self.code = code


class bm_params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("n_p", ctypes.c_uint32),
                ("alpha", ctypes.c_uint32), ("out_limbs", ctypes.c_uint32),
                ("q", ctypes.c_uint64 * 16), ("p", ctypes.c_uint64 * 4),
                ("scale", ctypes.c_double), ("sigma", ctypes.c_double), ("ring", ctypes.c_uint32)]

    @property
    def N(self):
        return 1 << self.log_n

    @property
    def slots(self):
        return self.N if self.ring == BM_RING_CI else self.N // 2

    def chain(self):
        return [int(self.q[i]) for i in range(self.n_q)]

    def special(self):
        return [int(self.p[i]) for i in range(self.n_p)]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_u32, _u64, _i32, _sz, _dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double

_SIGS = {
    "bm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "bm_last_error": (ctypes.c_char_p, [_P]),
    "bm_params_preset": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(bm_params)]),
    "bm_ctx_create": (ctypes.c_int, [ctypes.POINTER(bm_params), ctypes.c_int, _PP]),
    "bm_ctx_free": (None, [_P]),
    "bm_ctx_params": (ctypes.c_int, [_P, ctypes.POINTER(bm_params)]),
    "bm_ctx_set_group_chunk": (ctypes.c_int, [_P, _u32]),
    "bm_ctx_set_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "bm_ctx_pool_bytes": (ctypes.c_int, [_P, ctypes.POINTER(_u64)]),
    "bm_ctx_set_allocator": (ctypes.c_int, [_P, _P, _P, _P]),
    "bm_bench_modmul": (ctypes.c_int, [_P, _u32, _u32, _u32, _P, _P, _sz, ctypes.POINTER(_dbl)]),
    "bm_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "bm_profile_dump": (ctypes.c_int, [_P, ctypes.c_char_p, _sz, ctypes.POINTER(_sz)]),
    "bm_keygen": (ctypes.c_int, [_P, _u64, _P, _sz, _PP, _PP, _PP]),
    "bm_rotations_for": (ctypes.c_int, [_u32, _u32, _P, _sz, ctypes.POINTER(_sz)]),
    "bm_rotations_compress": (ctypes.c_int, [_u32, _u32, _P, _sz, ctypes.POINTER(_sz)]),
    "bm_rotations_hoisted": (ctypes.c_int, [_u32, _u32, _P, _sz, ctypes.POINTER(_sz)]),
    "bm_sk_export": (ctypes.c_int, [_P, _P, _sz]),
    "bm_pk_export": (ctypes.c_int, [_P, _u32, _P, _sz]),
    "bm_evk_export": (ctypes.c_int, [_P, _u64, _u32, _u32, _P, _sz]),
    "bm_pk_import": (ctypes.c_int, [_P, _P, _sz, _PP]),
    "bm_evk_import": (ctypes.c_int, [_P, _P, _sz, _P, _sz, _PP]),
    "bm_evk_galois": (ctypes.c_int, [_P, _P, _sz, ctypes.POINTER(_sz)]),
    "bm_sk_free": (None, [_P]),
    "bm_pk_free": (None, [_P]),
    "bm_evk_free": (None, [_P]),
    "bm_encode": (ctypes.c_int, [_P, _P, _sz, _dbl, _P]),
    "bm_encrypt_coeffs": (ctypes.c_int, [_P, _P, _P, _u32, _dbl, _u64, _u64, _PP]),
    "bm_encrypt_query": (ctypes.c_int, [_P, _P, _P, _u32, _u64, _u64, _PP]),
    "bm_encrypt_gallery": (ctypes.c_int, [_P, _P, _P, _u64, _u32, _u32, _u64, _u64, _PP]),
    "bm_gallery_import": (ctypes.c_int, [_P, _P, _u64, _u32, _u32, _u32, _dbl, _u64, _PP]),
    "bm_gallery_export": (ctypes.c_int, [_P, _P, _sz]),
    "bm_encrypt_template": (ctypes.c_int, [_P, _P, _P, _u32, _u64, _u64, _PP]),
    "bm_gallery_create": (ctypes.c_int, [_P, _u32, _u32, _u64, _u32, _PP]),
    "bm_enroll": (ctypes.c_int, [_P, _P, _P, _P, _P, _sz, _P, _P]),
    "bm_rotations_enroll": (ctypes.c_int, [_P, _u32, _u32, _P, _sz, ctypes.POINTER(_sz)]),
    "bm_gallery_info": (ctypes.c_int, [_P, ctypes.POINTER(_u64), ctypes.POINTER(_u32),
                                       ctypes.POINTER(_dbl)]),
    "bm_gallery_free": (None, [_P]),
    "bm_ct_import": (ctypes.c_int, [_P, _P, _u32, _u32, _dbl, _PP]),
    "bm_ct_export": (ctypes.c_int, [_P, _P, _sz]),
    "bm_ct_info": (ctypes.c_int, [_P, ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_dbl)]),
    "bm_ct_free": (None, [_P]),
    "bm_decrypt_slots": (ctypes.c_int, [_P, _P, _P, _P, _sz]),
    "bm_ntt": (ctypes.c_int, [_P, _P, _u32, _u32, _P, ctypes.c_int, _P]),
    "bm_op_add": (ctypes.c_int, [_P, _P, _P, _PP]),
    "bm_op_pmul": (ctypes.c_int, [_P, _P, _P, _dbl, _PP]),
    "bm_op_tensor": (ctypes.c_int, [_P, _P, _P, _PP]),
    "bm_op_relin": (ctypes.c_int, [_P, _P, _P, _PP]),
    "bm_op_rescale": (ctypes.c_int, [_P, _P, _PP]),
    "bm_op_rotate": (ctypes.c_int, [_P, _P, _P, _i32, _PP]),
    "bm_op_drop": (ctypes.c_int, [_P, _P, _u32, _PP]),
    "bm_masks_create": (ctypes.c_int, [_P, _u32, _u32, _PP]),
    "bm_masks_import": (ctypes.c_int, [_P, _u32, _u32, _P, _dbl, _PP]),
    "bm_masks_free": (None, [_P]),
    "bm_expand": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "bm_match": (ctypes.c_int, [_P, _P, _P, _P, _P, _u32, _u32, _P, _PP]),
    "bm_match_batch": (ctypes.c_int, [_P, _P, _P, _P, _sz, _u32, _u32, _P, _P]),
    "bm_match_noalloc": (ctypes.c_int, [_P, _P, _P, _u32, _dbl, _P, _P, _u32, _u32, _P, _sz, ctypes.POINTER(_sz),
                                        ctypes.POINTER(_dbl), _P]),
    "bm_autotune": (ctypes.c_int, [_P, _P, _P, _P, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_dbl)]),
    "bm_ctx_set_tuning": (ctypes.c_int, [_P, _P]),
    "bm_ctx_get_tuning": (ctypes.c_int, [_P, _P]),
    "bm_autotune_batch": (ctypes.c_int, [_P, _P, _P, _P, _sz, _P, _sz, _u32, ctypes.POINTER(_u32), _P,
                                         ctypes.POINTER(_dbl)]),
    "bm_result_info": (ctypes.c_int, [_P, ctypes.POINTER(_u64), ctypes.POINTER(_u32),
                                      ctypes.POINTER(_dbl)]),
    "bm_result_export": (ctypes.c_int, [_P, _u64, _P, _sz]),
    "bm_result_export_all": (ctypes.c_int, [_P, _P, _sz]),
    "bm_result_free": (None, [_P]),
    "bm_decrypt_scores": (ctypes.c_int, [_P, _P, _P, _P, _u64]),
    "bm_top1": (ctypes.c_int, [_P, _u64, _dbl, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_dbl)]),
    "bm_server_create": (ctypes.c_int, [_P, _P, _u64, _u32, _PP]),
    "bm_server_add_gallery": (ctypes.c_int, [_P, _P, ctypes.POINTER(_u32)]),
    "bm_server_submit": (ctypes.c_int, [_P, _u32, _P, ctypes.POINTER(_u64)]),
    "bm_server_poll": (ctypes.c_int, [_P, _u64, _PP]),
    "bm_server_drain": (ctypes.c_int, [_P]),
    "bm_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(_u64), ctypes.POINTER(_dbl),
                                       ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "bm_server_reset_stats": (ctypes.c_int, [_P]),
    "bm_server_free": (None, [_P]),
}

_lib = None


def _one_hip_runtime():
    """PyTorch ships its own HIP runtime (soname libamdhip64.so.7) and asks for
    it by the unversioned name.  Loaded first, it also serves this library, so
    the process holds one runtime and torch streams are valid stream handles
    here; loaded after the system runtime, torch would start a second one."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        _one_hip_runtime()
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libblindmatch.so is not built (run paper_2408_06167_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return sorted(_SIGS)


def _strerror(code):
    try:
        return lib().bm_strerror(code).decode()
    except Exception:
        return "status"


def _check(code, fn, ctx=None):
    if code != BM_OK:
        detail = lib().bm_last_error(ctx).decode(errors="replace") if _lib else ""
        raise BMError(code, fn, detail)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _out():
    return ctypes.c_void_p()


# ------------------------------------------------------------------ context and keys

def bm_params_preset(preset):
    p = bm_params()
    _check(lib().bm_params_preset(int(preset), ctypes.byref(p)), "bm_params_preset")
    return p


def bm_ctx_create(params, device=0):
    h = _out()
    _check(lib().bm_ctx_create(ctypes.byref(params), int(device), ctypes.byref(h)), "bm_ctx_create")
    return h


def bm_ctx_free(ctx):
    lib().bm_ctx_free(ctx)
    _alloc_hooks.pop(ctx.value, None)


def bm_ctx_params(ctx):
    p = bm_params()
    _check(lib().bm_ctx_params(ctx, ctypes.byref(p)), "bm_ctx_params", ctx)
    return p


def bm_ctx_set_group_chunk(ctx, groups):
    _check(lib().bm_ctx_set_group_chunk(ctx, int(groups)), "bm_ctx_set_group_chunk", ctx)


def bm_ctx_set_graphs(ctx, on=True):
    _check(lib().bm_ctx_set_graphs(ctx, 1 if on else 0), "bm_ctx_set_graphs", ctx)


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
# context address -> every callback pair it was given; blocks keep the
# allocator they came from, so all pairs stay alive until bm_ctx_free
_alloc_hooks = {}


def bm_ctx_set_allocator(ctx, alloc=None, free=None):
    """Device memory of the context from alloc(nbytes) -> device address (0 when
    it cannot), returned through free(address); both None restores hipMalloc.
    An exception in a callback is printed and counts as a failed allocation."""
    if alloc is None and free is None:
        a = f = None
    else:
        def _a(n, _user, _fn=alloc):
            return int(_fn(int(n)) or 0) if _fn else 0

        def _f(ptr, _user, _fn=free):
            if _fn:
                _fn(int(ptr))
        cbs = (_ALLOC_FN(_a), _FREE_FN(_f))
        _alloc_hooks.setdefault(ctx.value, []).append(cbs)
        a = ctypes.cast(cbs[0], ctypes.c_void_p) if alloc else None
        f = ctypes.cast(cbs[1], ctypes.c_void_p) if free else None
    _check(lib().bm_ctx_set_allocator(ctx, a, f, None), "bm_ctx_set_allocator", ctx)


def torch_allocator(device=0):
    """(alloc, free) over torch's caching allocator on `device` (current stream),
    for bm_ctx_set_allocator."""
    import torch

    def alloc(n):
        return torch.cuda.caching_allocator_alloc(n, device)

    def free(ptr):
        torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


def bm_ctx_pool_bytes(ctx):
    v = _u64()
    _check(lib().bm_ctx_pool_bytes(ctx, ctypes.byref(v)), "bm_ctx_pool_bytes", ctx)
    return int(v.value)


def bm_profile_enable(ctx, on=True):
    _check(lib().bm_profile_enable(ctx, 1 if on else 0), "bm_profile_enable", ctx)


def bm_bench_modmul(ctx, prime, blocks, iters, seed, n_words=0):
    """(kernel ms, first n_words output words) of the butterfly issue-rate probe."""
    sd = np.ascontiguousarray(seed, dtype=np.uint64)
    if sd.shape != (24,):
        raise ValueError("seed must hold 24 residues")
    w = np.zeros(max(int(n_words), 1), dtype=np.uint64)
    ms = _dbl()
    _check(lib().bm_bench_modmul(ctx, int(prime), int(blocks), int(iters), _ptr(sd), _ptr(w), int(n_words),
                                 ctypes.byref(ms)), "bm_bench_modmul", ctx)
    return float(ms.value), w[:int(n_words)]


def bm_profile_dump(ctx):
    """{kernel: dict(launches, ms, bytes, ops)} since bm_profile_enable."""
    need = _sz()
    _check(lib().bm_profile_dump(ctx, None, 0, ctypes.byref(need)), "bm_profile_dump", ctx)
    buf = ctypes.create_string_buffer(need.value + 1)
    _check(lib().bm_profile_dump(ctx, buf, need.value + 1, ctypes.byref(need)), "bm_profile_dump", ctx)
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms, b, o = line.rsplit(None, 4)        # kernel names hold spaces
        out[name] = dict(launches=int(n), ms=float(ms), bytes=float(b), ops=float(o))
    return out


def bm_rotations_for(d, k):
    n = _sz()
    _check(lib().bm_rotations_for(int(d), int(k), None, 0, ctypes.byref(n)), "bm_rotations_for")
    out = np.zeros(n.value, dtype=np.int32)
    _check(lib().bm_rotations_for(int(d), int(k), _ptr(out), out.size, ctypes.byref(n)), "bm_rotations_for")
    return [int(x) for x in out]


def bm_rotations_hoisted(d, k):
    n = _sz(0)
    _check(lib().bm_rotations_hoisted(int(d), int(k), None, 0, ctypes.byref(n)), "bm_rotations_hoisted")
    out = np.zeros(n.value, dtype=np.int32)
    _check(lib().bm_rotations_hoisted(int(d), int(k), _ptr(out), out.size, ctypes.byref(n)),
           "bm_rotations_hoisted")
    return [int(v) for v in out]


def bm_rotations_compress(d, k):
    n = _sz(0)
    _check(lib().bm_rotations_compress(int(d), int(k), None, 0, ctypes.byref(n)), "bm_rotations_compress")
    out = np.zeros(n.value, dtype=np.int32)
    _check(lib().bm_rotations_compress(int(d), int(k), _ptr(out), out.size, ctypes.byref(n)),
           "bm_rotations_compress")
    return [int(v) for v in out]


def bm_keygen(ctx, seed, rotations=()):
    rots = np.ascontiguousarray(sorted(set(int(r) for r in rotations)), dtype=np.int32)
    sk, pk, evk = _out(), _out(), _out()
    _check(lib().bm_keygen(ctx, int(seed), _ptr(rots) if rots.size else None, rots.size,
                           ctypes.byref(sk), ctypes.byref(pk), ctypes.byref(evk)), "bm_keygen", ctx)
    return sk, pk, evk


def bm_sk_export(sk, N):
    s = np.zeros(N, dtype=np.int64)
    _check(lib().bm_sk_export(sk, _ptr(s), N), "bm_sk_export")
    return s


def bm_pk_export(ctx, pk, comp, limbs, N):
    w = np.zeros((limbs, N), dtype=np.uint64)
    _check(lib().bm_pk_export(pk, int(comp), _ptr(w), w.size), "bm_pk_export", ctx)
    return w


def bm_evk_export(ctx, evk, galois, digit, comp, nprimes, N):
    w = np.zeros((nprimes, N), dtype=np.uint64)
    _check(lib().bm_evk_export(evk, int(galois), int(digit), int(comp), _ptr(w), w.size),
           "bm_evk_export", ctx)
    return w


def bm_pk_import(ctx, words):
    """words: [2][L+1][N] uint64 coefficient-domain public key (b, a)."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    h = _out()
    _check(lib().bm_pk_import(ctx, _ptr(w), w.size, ctypes.byref(h)), "bm_pk_import", ctx)
    return h


def bm_evk_import(ctx, galois, words):
    """words: [1 + len(galois)][dnum][2][L+1+K][N] uint64: the relinearisation
    key, then the Galois key of each element in `galois`."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    g = np.ascontiguousarray(galois, dtype=np.uint64)
    h = _out()
    _check(lib().bm_evk_import(ctx, _ptr(g) if g.size else None, g.size, _ptr(w), w.size, ctypes.byref(h)),
           "bm_evk_import", ctx)
    return h


def bm_evk_galois(evk):
    n = _sz(0)
    _check(lib().bm_evk_galois(evk, None, 0, ctypes.byref(n)), "bm_evk_galois")
    g = np.zeros(n.value, dtype=np.uint64)
    _check(lib().bm_evk_galois(evk, _ptr(g) if g.size else None, g.size, ctypes.byref(n)), "bm_evk_galois")
    return [int(x) for x in g]


def bm_sk_free(h):
    lib().bm_sk_free(h)


def bm_pk_free(h):
    lib().bm_pk_free(h)


def bm_evk_free(h):
    lib().bm_evk_free(h)


# ------------------------------------------------------------------ encode / encrypt

def bm_encode(ctx, slots, scale):
    slots = np.ascontiguousarray(slots, dtype=np.float64)
    out = np.zeros(bm_ctx_params(ctx).N, dtype=np.int64)
    _check(lib().bm_encode(ctx, _ptr(slots), slots.size, float(scale), _ptr(out)), "bm_encode", ctx)
    return out


def bm_encrypt_coeffs(ctx, pk, coeffs, limbs, scale, seed, ct_id):
    m = np.ascontiguousarray(coeffs, dtype=np.int64)
    h = _out()
    _check(lib().bm_encrypt_coeffs(ctx, pk, _ptr(m), int(limbs), float(scale), int(seed), int(ct_id),
                                   ctypes.byref(h)), "bm_encrypt_coeffs", ctx)
    return h


def bm_encrypt_query(ctx, pk, q, seed, ct_id):
    q = np.ascontiguousarray(q, dtype=np.float32)
    h = _out()
    _check(lib().bm_encrypt_query(ctx, pk, _ptr(q), q.size, int(seed), int(ct_id), ctypes.byref(h)),
           "bm_encrypt_query", ctx)
    return h


def bm_encrypt_gallery(ctx, pk, X, k, seed, ct_id_base):
    X = np.ascontiguousarray(X, dtype=np.float32)
    h = _out()
    _check(lib().bm_encrypt_gallery(ctx, pk, _ptr(X), X.shape[0], X.shape[1], int(k), int(seed),
                                    int(ct_id_base), ctypes.byref(h)), "bm_encrypt_gallery", ctx)
    return h


def bm_gallery_import(ctx, words, d, k, limbs, scale, n_templates):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    groups = w.shape[0]
    h = _out()
    _check(lib().bm_gallery_import(ctx, _ptr(w), groups, int(d), int(k), int(limbs), float(scale),
                                   int(n_templates), ctypes.byref(h)), "bm_gallery_import", ctx)
    return h


def bm_encrypt_template(ctx, pk, x, seed, ct_id):
    x = np.ascontiguousarray(x, dtype=np.float32)
    h = _out()
    _check(lib().bm_encrypt_template(ctx, pk, _ptr(x), x.size, int(seed), int(ct_id), ctypes.byref(h)),
           "bm_encrypt_template", ctx)
    return h


def bm_gallery_create(ctx, d, k, n_templates, limbs):
    h = _out()
    _check(lib().bm_gallery_create(ctx, int(d), int(k), int(n_templates), int(limbs), ctypes.byref(h)),
           "bm_gallery_create", ctx)
    return h


def bm_enroll(ctx, evk, gallery, users, indices, masks=None, stream=None):
    n = len(users)
    ua = (ctypes.c_void_p * max(n, 1))(*[u.value for u in users])
    idx = np.ascontiguousarray(indices, dtype=np.uint64)
    assert idx.size == n
    _check(lib().bm_enroll(ctx, evk, gallery, ctypes.cast(ua, _P), _ptr(idx), n, masks,
                           ctypes.c_void_p(stream) if stream else None), "bm_enroll", ctx)


def bm_rotations_enroll(ctx, d, k):
    n = _sz(0)
    _check(lib().bm_rotations_enroll(ctx, int(d), int(k), None, 0, ctypes.byref(n)), "bm_rotations_enroll")
    out = np.zeros(n.value, dtype=np.int32)
    _check(lib().bm_rotations_enroll(ctx, int(d), int(k), _ptr(out), out.size, ctypes.byref(n)),
           "bm_rotations_enroll")
    return [int(v) for v in out]


def bm_gallery_info(g):
    G, l, s = _u64(), _u32(), _dbl()
    _check(lib().bm_gallery_info(g, ctypes.byref(G), ctypes.byref(l), ctypes.byref(s)), "bm_gallery_info")
    return int(G.value), int(l.value), float(s.value)


def bm_gallery_export(ctx, g, k, N):
    G, l, _ = bm_gallery_info(g)
    w = np.zeros((G, k, 2, l, N), dtype=np.uint64)
    _check(lib().bm_gallery_export(g, _ptr(w), w.size), "bm_gallery_export", ctx)
    return w


def bm_gallery_free(g):
    lib().bm_gallery_free(g)


# ------------------------------------------------------------------ ciphertexts

def bm_ct_import(ctx, words, scale):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    comps, limbs = w.shape[0], w.shape[1]
    h = _out()
    _check(lib().bm_ct_import(ctx, _ptr(w), comps, limbs, float(scale), ctypes.byref(h)),
           "bm_ct_import", ctx)
    return h


def bm_ct_info(ct):
    c, l, s = _u32(), _u32(), _dbl()
    _check(lib().bm_ct_info(ct, ctypes.byref(c), ctypes.byref(l), ctypes.byref(s)), "bm_ct_info")
    return int(c.value), int(l.value), float(s.value)


def bm_ct_export(ctx, ct, N):
    comps, limbs, scale = bm_ct_info(ct)
    w = np.zeros((comps, limbs, N), dtype=np.uint64)
    _check(lib().bm_ct_export(ct, _ptr(w), w.size), "bm_ct_export", ctx)
    return w, scale


def bm_ct_free(ct):
    lib().bm_ct_free(ct)


def bm_decrypt_slots(ctx, sk, ct, n):
    out = np.zeros(n, dtype=np.float64)
    _check(lib().bm_decrypt_slots(ctx, sk, ct, _ptr(out), n), "bm_decrypt_slots", ctx)
    return out


# ------------------------------------------------------------------ primitive operations

def bm_ntt(ctx, dev_ptr, n_polys, prime_ids, inverse, stream=None):
    ids = np.ascontiguousarray(prime_ids, dtype=np.uint32)
    _check(lib().bm_ntt(ctx, ctypes.c_void_p(dev_ptr), int(n_polys), ids.size, _ptr(ids),
                        1 if inverse else 0, ctypes.c_void_p(stream) if stream else None),
           "bm_ntt", ctx)


def _op(name, ctx, *args):
    h = _out()
    _check(getattr(lib(), name)(ctx, *args, ctypes.byref(h)), name, ctx)
    return h


def bm_op_add(ctx, a, b):
    return _op("bm_op_add", ctx, a, b)


def bm_op_pmul(ctx, a, pt, pt_scale):
    pt = np.ascontiguousarray(pt, dtype=np.int64)
    return _op("bm_op_pmul", ctx, a, _ptr(pt), float(pt_scale))


def bm_op_tensor(ctx, a, b):
    return _op("bm_op_tensor", ctx, a, b)


def bm_op_relin(ctx, evk, a):
    return _op("bm_op_relin", ctx, evk, a)


def bm_op_rescale(ctx, a):
    return _op("bm_op_rescale", ctx, a)


def bm_op_rotate(ctx, evk, a, r):
    return _op("bm_op_rotate", ctx, evk, a, int(r))


def bm_op_drop(ctx, a, limbs):
    return _op("bm_op_drop", ctx, a, int(limbs))


# ------------------------------------------------------------------ Blind-Match

def bm_masks_create(ctx, d, k):
    return _op("bm_masks_create", ctx, int(d), int(k))


def bm_masks_import(ctx, d, k, coeffs, scale):
    c = np.ascontiguousarray(coeffs, dtype=np.int64)
    return _op("bm_masks_import", ctx, int(d), int(k), _ptr(c), float(scale))


def bm_masks_free(m):
    lib().bm_masks_free(m)


def bm_expand(ctx, evk, q, masks, k):
    outs = (ctypes.c_void_p * k)()
    _check(lib().bm_expand(ctx, evk, q, masks, ctypes.cast(outs, _P)), "bm_expand", ctx)
    return [ctypes.c_void_p(outs[i]) for i in range(k)]


def bm_match(ctx, evk, q, gallery, masks=None, schedule=BM_S1, out_limbs=0, stream=None):
    return _op("bm_match", ctx, evk, q, gallery, masks, int(schedule), int(out_limbs),
               ctypes.c_void_p(stream) if stream else None)


def bm_match_noalloc(ctx, evk, q_ptr, q_limbs, q_scale, g, masks=None, schedule=BM_S2, out_limbs=0, out_ptr=None,
                     n_out_words=0, stream=None):
    """bm_match on device buffers (integer addresses) with the library's
    scratch array; returns (words the output needs, result scale).  With
    out_ptr None only the size is reported."""
    needed, sc = _sz(0), _dbl(0)
    _check(lib().bm_match_noalloc(ctx, evk, ctypes.c_void_p(q_ptr), int(q_limbs), float(q_scale), g, masks,
                                  int(schedule), int(out_limbs), ctypes.c_void_p(out_ptr) if out_ptr else None,
                                  int(n_out_words), ctypes.byref(needed), ctypes.byref(sc),
                                  ctypes.c_void_p(stream) if stream else None), "bm_match_noalloc", ctx)
    return needed.value, sc.value


def bm_match_batch(ctx, evk, queries, galleries, schedule=BM_S1, out_limbs=0, stream=None):
    n = len(queries)
    qa = (ctypes.c_void_p * n)(*[q.value for q in queries])
    ga = (ctypes.c_void_p * n)(*[g.value for g in galleries])
    outs = (ctypes.c_void_p * n)()
    _check(lib().bm_match_batch(ctx, evk, ctypes.cast(qa, _P), ctypes.cast(ga, _P), n, int(schedule),
                                int(out_limbs), ctypes.c_void_p(stream) if stream else None,
                                ctypes.cast(outs, _P)), "bm_match_batch", ctx)
    return [ctypes.c_void_p(outs[i]) for i in range(n)]


class bm_tuning(ctypes.Structure):
    _fields_ = [("group_chunk", ctypes.c_uint32), ("kip_variant", ctypes.c_uint32),
                ("ntt_row_views", ctypes.c_uint32), ("kip_order", ctypes.c_uint32),
                ("fused_occupancy", ctypes.c_uint32), ("column_sources", ctypes.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def bm_ctx_set_tuning(ctx, group_chunk=0, kip_variant=0, ntt_row_views=0, kip_order=0, fused_occupancy=0,
                      column_sources=0):
    t = bm_tuning(int(group_chunk), int(kip_variant), int(ntt_row_views), int(kip_order), int(fused_occupancy),
                  int(column_sources))
    _check(lib().bm_ctx_set_tuning(ctx, ctypes.byref(t)), "bm_ctx_set_tuning", ctx)


def bm_ctx_get_tuning(ctx):
    t = bm_tuning()
    _check(lib().bm_ctx_get_tuning(ctx, ctypes.byref(t)), "bm_ctx_get_tuning", ctx)
    return t.as_dict()


def bm_autotune_batch(ctx, evk, qs, gs, schedules, out_limbs=0):
    """Returns (schedule, tuning dict, ms per batch); the knobs stay set."""
    n = len(qs)
    qa = (ctypes.c_void_p * n)(*[q.value for q in qs])
    ga = (ctypes.c_void_p * n)(*[g.value for g in gs])
    sa = (_u32 * len(schedules))(*[int(x) for x in schedules])
    bs, t, ms = _u32(0), bm_tuning(), _dbl(0)
    _check(lib().bm_autotune_batch(ctx, evk, ctypes.cast(qa, _P), ctypes.cast(ga, _P), n, ctypes.cast(sa, _P),
                                   len(schedules), int(out_limbs), ctypes.byref(bs), ctypes.byref(t),
                                   ctypes.byref(ms)), "bm_autotune_batch", ctx)
    return bs.value, t.as_dict(), ms.value


def bm_autotune(ctx, evk, q, gallery, schedule=BM_S2):
    """(best group_chunk, ms per match); the context keeps the best chunk."""
    c, ms = _u32(), _dbl()
    _check(lib().bm_autotune(ctx, evk, q, gallery, int(schedule), ctypes.byref(c), ctypes.byref(ms)),
           "bm_autotune", ctx)
    return int(c.value), float(ms.value)


def bm_result_info(r):
    G, l, s = _u64(), _u32(), _dbl()
    _check(lib().bm_result_info(r, ctypes.byref(G), ctypes.byref(l), ctypes.byref(s)), "bm_result_info")
    return int(G.value), int(l.value), float(s.value)


def bm_result_export(ctx, r, group, N):
    _, limbs, scale = bm_result_info(r)
    w = np.zeros((2, limbs, N), dtype=np.uint64)
    _check(lib().bm_result_export(r, int(group), _ptr(w), w.size), "bm_result_export", ctx)
    return w, scale


def bm_result_export_all(ctx, r, N):
    """words[groups][2][limbs][N] of every result ciphertext, and the scale."""
    groups, limbs, scale = bm_result_info(r)
    w = np.zeros((groups, 2, limbs, N), dtype=np.uint64)
    _check(lib().bm_result_export_all(r, _ptr(w), w.size), "bm_result_export_all", ctx)
    return w, scale


def bm_result_free(r):
    lib().bm_result_free(r)


def bm_decrypt_scores(ctx, sk, r, n):
    out = np.zeros(n, dtype=np.float64)
    _check(lib().bm_decrypt_scores(ctx, sk, r, _ptr(out), int(n)), "bm_decrypt_scores", ctx)
    return out


def bm_top1(scores, threshold=float("-inf")):
    s = np.ascontiguousarray(scores, dtype=np.float64)
    idx, best = ctypes.c_int64(), _dbl()
    _check(lib().bm_top1(_ptr(s), s.size, float(threshold), ctypes.byref(idx), ctypes.byref(best)), "bm_top1")
    return int(idx.value), float(best.value)


# ------------------------------------------------------------------ serving

def bm_server_create(ctx, evk, hbm_budget_bytes, schedule=BM_S2):
    return _op("bm_server_create", ctx, evk, int(hbm_budget_bytes), int(schedule))


def bm_server_add_gallery(server, gallery):
    gid = _u32()
    _check(lib().bm_server_add_gallery(server, gallery, ctypes.byref(gid)), "bm_server_add_gallery")
    return int(gid.value)


def bm_server_submit(server, gallery_id, q):
    t = _u64()
    _check(lib().bm_server_submit(server, int(gallery_id), q, ctypes.byref(t)), "bm_server_submit")
    return int(t.value)


def bm_server_poll(server, ticket):
    h = _out()
    _check(lib().bm_server_poll(server, int(ticket), ctypes.byref(h)), "bm_server_poll")
    return h if h.value else None


def bm_server_drain(server):
    _check(lib().bm_server_drain(server), "bm_server_drain")


def bm_server_stats(server):
    n, p50, p99, mb = _u64(), _dbl(), _dbl(), _dbl()
    _check(lib().bm_server_stats(server, ctypes.byref(n), ctypes.byref(p50), ctypes.byref(p99),
                                 ctypes.byref(mb)), "bm_server_stats")
    return dict(completed=int(n.value), p50_ms=p50.value, p99_ms=p99.value, mean_batch=mb.value)


def bm_server_reset_stats(server):
    _check(lib().bm_server_reset_stats(server), "bm_server_reset_stats")


def bm_server_free(server):
    lib().bm_server_free(server)
