"""Drive the library's call sequences with BM_DRY_RUN=1 (no GPU): every kernel
launch is checked against the buffers it would touch, none is executed.
Run as a script by test_dry_run.py; exits non-zero on the first failure."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
assert os.environ.get("BM_DRY_RUN") == "1"
import paper_2408_06167_amd as bm  # noqa: E402


def flow(preset, shapes, n_templates, hook=None):
    p = bm.bm_params_preset(preset)
    ctx = bm.bm_ctx_create(p, 0)
    if hook:
        bm.bm_ctx_set_allocator(ctx, *hook)
    # the butterfly issue-rate probe, all of its output copied back
    bm.bm_bench_modmul(ctx, p.n_q, 2, 4, np.arange(24, dtype=np.uint64), 2 * 256 * 16)
    N, L1 = p.N, p.n_q
    rots = set()
    for d, k in shapes:
        rots.update(bm.bm_rotations_for(d, k))
        rots.update(bm.bm_rotations_compress(d, k))
        rots.update(bm.bm_rotations_enroll(ctx, d, k))
        if d // k <= 32:
            rots.update(bm.bm_rotations_hoisted(d, k))
    sk, pk, evk = bm.bm_keygen(ctx, 1, sorted(rots))
    rng = np.random.default_rng(0)
    words = rng.integers(0, 1 << 40, size=(2, L1, N), dtype=np.uint64)
    a = bm.bm_ct_import(ctx, words, p.scale)
    b = bm.bm_ct_import(ctx, words, p.scale)
    for op in (lambda: bm.bm_op_add(ctx, a, b), lambda: bm.bm_op_tensor(ctx, a, b),
               lambda: bm.bm_op_rescale(ctx, a), lambda: bm.bm_op_drop(ctx, a, 1),
               lambda: bm.bm_op_pmul(ctx, a, np.ones(N, dtype=np.int64), 2.0)):
        bm.bm_ct_free(op())
    t = bm.bm_op_tensor(ctx, a, b)
    bm.bm_ct_free(bm.bm_op_relin(ctx, evk, t))
    for r in sorted(rots)[:3]:
        bm.bm_ct_free(bm.bm_op_rotate(ctx, evk, a, r))
    for limbs in range(1, L1 + 1):
        c = bm.bm_encrypt_coeffs(ctx, pk, np.zeros(N, dtype=np.int64), limbs, p.scale, 1, limbs)
        bm.bm_ct_export(ctx, c, N)
        if limbs >= 2:
            bm.bm_ct_free(bm.bm_op_rescale(ctx, c))
            bm.bm_ct_free(bm.bm_op_rotate(ctx, evk, c, sorted(rots)[-1]))
        bm.bm_ct_free(c)
    for d, k in shapes:
        X = rng.standard_normal((n_templates, d)).astype(np.float32)
        q = bm.bm_encrypt_query(ctx, pk, X[0], 1, 1)
        g = bm.bm_encrypt_gallery(ctx, pk, X, k, 1, 10)
        if k > 1:
            m = bm.bm_masks_create(ctx, d, k)
            for h in bm.bm_expand(ctx, evk, q, m, k):
                bm.bm_ct_free(h)
            bm.bm_masks_free(m)
        for s in (1, 2, 1 | bm.BM_LEVEL_MIN, 2 | bm.BM_LEVEL_MIN):
            bm.bm_ctx_set_graphs(ctx, (s & 2) != 0)
            for chunk in (0, 1, 3):
                bm.bm_ctx_set_group_chunk(ctx, chunk)
                r = bm.bm_match(ctx, evk, q, g, None, schedule=s, out_limbs=0)
                bm.bm_decrypt_scores(ctx, sk, r, n_templates)
                G, limbs, _ = bm.bm_result_info(r)
                bm.bm_result_export(ctx, r, G - 1, N)
                bm.bm_result_export_all(ctx, r, N)
                bm.bm_result_free(r)
        # compression: needs one level more than the plain match
        can_compress = preset in (2, 4) or k == 1
        if d // k <= 32:
            for s in (1 | bm.BM_HOIST, 2 | bm.BM_HOIST | bm.BM_LEVEL_MIN):
                for graphs in (False, True):
                    bm.bm_ctx_set_graphs(ctx, graphs)
                    r = bm.bm_match(ctx, evk, q, g, None, schedule=s, out_limbs=0)
                    bm.bm_decrypt_scores(ctx, sk, r, n_templates)
                    bm.bm_result_free(r)
        for s in (2 | bm.BM_COMPRESS, 1 | bm.BM_LEVEL_MIN | bm.BM_COMPRESS):
            bm.bm_ctx_set_graphs(ctx, (s & 2) != 0)
            try:
                r = bm.bm_match(ctx, evk, q, g, None, schedule=s, out_limbs=0)
            except bm.BMError as e:
                assert not can_compress and e.code == bm.BM_ELEVEL, e
                continue
            assert can_compress
            bm.bm_decrypt_scores(ctx, sk, r, n_templates)
            G, limbs, _ = bm.bm_result_info(r)
            bm.bm_result_export(ctx, r, G - 1, N)
            bm.bm_result_free(r)
        bm.bm_ctx_set_graphs(ctx, False)
        if can_compress:
            for r in bm.bm_match_batch(ctx, evk, [q, q, q], [g, g, g], schedule=2 | bm.BM_COMPRESS):
                bm.bm_result_free(r)
        rs = bm.bm_match_batch(ctx, evk, [q, q, q], [g, g, g], schedule=2)
        for r in rs:
            bm.bm_result_free(r)
        rs = bm.bm_match_batch(ctx, evk, [q, q], [g, g], schedule=2 | bm.BM_LEVEL_MIN)
        bm.bm_autotune(ctx, evk, q, g, 2)
        for r in rs:
            bm.bm_result_free(r)
        bm.bm_ctx_set_group_chunk(ctx, 0)
        # server-side enrollment into an empty gallery, then a match against it
        c_, T_ = d // k, p.slots // (d // k)
        eg = bm.bm_gallery_create(ctx, d, k, 2 * T_, L1 - 1)
        users = [bm.bm_encrypt_template(ctx, pk, X[i], 1, 700 + i) for i in range(3)]
        bm.bm_enroll(ctx, evk, eg, users, [0, T_ + 1, 2 * T_ - 1])
        for u in users:
            bm.bm_ct_free(u)
        r = bm.bm_match(ctx, evk, q, eg, None, schedule=2, out_limbs=0)
        bm.bm_decrypt_scores(ctx, sk, r, 2 * T_)
        bm.bm_result_free(r)
        bm.bm_gallery_free(eg)
        srv = bm.bm_server_create(ctx, evk, 64 << 30, 2 | (bm.BM_LEVEL_MIN if k > 1 else 0) |
                                  (bm.BM_COMPRESS if can_compress and k != 4 else 0))
        gid = bm.bm_server_add_gallery(srv, g)
        tickets = [bm.bm_server_submit(srv, gid, bm.bm_encrypt_query(ctx, pk, X[i], 1, 100 + i))
                   for i in range(5)]
        bm.bm_server_drain(srv)
        for t_ in tickets:
            bm.bm_result_free(bm.bm_server_poll(srv, t_))
        bm.bm_server_free(srv)
        bm.bm_ct_free(q)
        print("preset %d d=%d k=%d ok" % (preset, d, k), flush=True)
    for h in (a, b, t):
        bm.bm_ct_free(h)
    bm.bm_sk_free(sk)
    bm.bm_pk_free(pk)
    bm.bm_evk_free(evk)
    bm.bm_ctx_free(ctx)


class HostAllocator:
    """Caller allocator over libc malloc (device memory is host memory in a dry
    run) that records every block it hands out."""

    def __init__(self):
        self.libc = ctypes.CDLL(None)
        self.libc.malloc.restype = ctypes.c_void_p
        self.libc.malloc.argtypes = [ctypes.c_size_t]
        self.libc.free.argtypes = [ctypes.c_void_p]
        self.live, self.allocs, self.frees = {}, 0, 0

    def alloc(self, n):
        ptr = self.libc.malloc(n)
        assert ptr not in self.live
        self.live[ptr] = n
        self.allocs += 1
        return ptr

    def free(self, ptr):
        assert ptr in self.live, "block freed that this allocator did not hand out"
        del self.live[ptr]
        self.frees += 1
        self.libc.free(ptr)


def allocator_hook_flow():
    # a whole flow (graphs, batches, enrollment, server lanes) on a caller's allocator
    h = HostAllocator()
    flow(1, [(16, 1), (16, 4)], 300, hook=(h.alloc, h.free))
    assert h.allocs > 0 and h.frees == h.allocs and not h.live, (h.allocs, h.frees, len(h.live))
    # switching allocators: blocks in use go back to the one they came from
    h1, h2 = HostAllocator(), HostAllocator()
    p = bm.bm_params_preset(1)
    ctx = bm.bm_ctx_create(p, 0)
    bm.bm_ctx_set_allocator(ctx, h1.alloc, h1.free)
    sk, pk, evk = bm.bm_keygen(ctx, 1, bm.bm_rotations_for(16, 1))
    held = bm.bm_ctx_pool_bytes(ctx)
    assert h1.allocs > 0 and sum(h1.live.values()) == held, (sum(h1.live.values()), held)
    bm.bm_ctx_set_allocator(ctx, h2.alloc, h2.free)
    q = bm.bm_encrypt_query(ctx, pk, np.ones(16, dtype=np.float32), 1, 1)
    assert h2.allocs > 0
    bm.bm_ctx_set_allocator(ctx)           # back to the library's own allocation
    g = bm.bm_encrypt_gallery(ctx, pk, np.ones((20, 16), dtype=np.float32), 1, 1, 10)
    bm.bm_result_free(bm.bm_match(ctx, evk, q, g, None, schedule=1))
    for f, x in ((bm.bm_gallery_free, g), (bm.bm_ct_free, q), (bm.bm_sk_free, sk), (bm.bm_pk_free, pk),
                 (bm.bm_evk_free, evk)):
        f(x)
    try:
        bm.bm_ctx_set_allocator(ctx, h1.alloc, None)
        raise AssertionError("one missing callback accepted")
    except bm.BMError as e:
        assert e.code == bm.BM_EINVAL
    bm.bm_ctx_free(ctx)
    for h in (h1, h2):
        assert h.frees == h.allocs and not h.live, (h.allocs, h.frees)
    print("allocator hook ok", flush=True)


def input_checks():
    """Host-side rejection of inputs the method cannot take, each with the
    status the header states."""
    p = bm.bm_params_preset(1)
    ctx = bm.bm_ctx_create(p, 0)
    sk, pk, evk = bm.bm_keygen(ctx, 1, bm.bm_rotations_for(16, 1))

    def status(f):
        try:
            f()
        except bm.BMError as e:
            return e.code
        return bm.BM_OK
    X = np.ones((10, 16), dtype=np.float32)
    one = lambda d: np.ones(d, dtype=np.float32)   # noqa: E731
    q16 = bm.bm_encrypt_query(ctx, pk, one(16), 1, 1)
    q8 = bm.bm_encrypt_query(ctx, pk, one(8), 1, 2)
    g = bm.bm_encrypt_gallery(ctx, pk, X, 1, 1, 10)
    w = np.zeros((2, p.n_q, p.N), dtype=np.uint64)
    a = bm.bm_ct_import(ctx, w, p.scale)
    b = bm.bm_ct_import(ctx, w, 2 * p.scale)
    c2 = bm.bm_ct_import(ctx, w[:, :2], p.scale)
    c1 = bm.bm_ct_import(ctx, w[:, :1], p.scale)
    r = bm.bm_match(ctx, evk, q16, g, None, schedule=1)
    cases = [
        ("empty gallery", lambda: bm.bm_encrypt_gallery(ctx, pk, np.ones((0, 16), dtype=np.float32), 1, 1, 10),
         bm.BM_EINVAL),
        ("d = 0", lambda: bm.bm_encrypt_query(ctx, pk, one(0), 1, 1), bm.BM_EDIM),
        ("d not a power of two", lambda: bm.bm_encrypt_query(ctx, pk, one(24), 1, 1), bm.BM_EDIM),
        ("d above the slots", lambda: bm.bm_encrypt_query(ctx, pk, one(2 * p.slots), 1, 1), bm.BM_EDIM),
        ("k not a power of two", lambda: bm.bm_encrypt_gallery(ctx, pk, X, 3, 1, 10), bm.BM_EDIM),
        ("k above d", lambda: bm.bm_encrypt_gallery(ctx, pk, X, 32, 1, 10), bm.BM_EDIM),
        ("query d != gallery d", lambda: bm.bm_match(ctx, evk, q8, g, None, schedule=1), bm.BM_EDIM),
        ("query d != gallery d, batched", lambda: bm.bm_match_batch(ctx, evk, [q16, q8], [g, g], schedule=1),
         bm.BM_EDIM),
        ("expansion with masks of another d", lambda: bm.bm_expand(ctx, evk, q8, bm.bm_masks_create(ctx, 16, 2), 2),
         bm.BM_EDIM),
        ("schedule without S1 or S2", lambda: bm.bm_match(ctx, evk, q16, g, None, schedule=0), bm.BM_EINVAL),
        ("S1 and S2 together", lambda: bm.bm_match(ctx, evk, q16, g, None, schedule=3), bm.BM_EINVAL),
        ("query below the gallery level", lambda: bm.bm_match(ctx, evk, c1, g, None, schedule=1), bm.BM_ELEVEL),
        ("decrypt with another template count", lambda: bm.bm_decrypt_scores(ctx, sk, r, 11), bm.BM_EINVAL),
        ("export of a missing group", lambda: bm.bm_result_export(ctx, r, 5, p.N), bm.BM_EINVAL),
        ("add at different scales", lambda: bm.bm_op_add(ctx, a, b), bm.BM_ESCALE),
        ("add at different levels", lambda: bm.bm_op_add(ctx, a, c2), bm.BM_ELEVEL),
        ("rotation without its key", lambda: bm.bm_op_rotate(ctx, evk, a, 3), bm.BM_ENOKEY),
        ("rescale of one limb", lambda: bm.bm_op_rescale(ctx, c1), bm.BM_ELEVEL),
        ("top-1 of no scores", lambda: bm.bm_top1(np.zeros(0)), bm.BM_EINVAL),
        ("fused occupancy 5", lambda: bm.bm_ctx_set_tuning(ctx, fused_occupancy=5), bm.BM_EINVAL),
        ("column sources 2", lambda: bm.bm_ctx_set_tuning(ctx, column_sources=2), bm.BM_EINVAL),
        ("key inner product order 4", lambda: bm.bm_ctx_set_tuning(ctx, kip_order=4), bm.BM_EINVAL),
    ]
    # handles of another context (its buffers are sized for its own ring)
    ctx2 = bm.bm_ctx_create(bm.bm_params_preset(3), 0)
    sk2, pk2, evk2 = bm.bm_keygen(ctx2, 1, bm.bm_rotations_for(16, 1))
    q2 = bm.bm_encrypt_query(ctx2, pk2, one(16), 1, 1)
    cases += [
        ("query of another context", lambda: bm.bm_match(ctx, evk, q2, g, None, schedule=1), bm.BM_EINVAL),
        ("keys of another context", lambda: bm.bm_match(ctx, evk2, q16, g, None, schedule=1), bm.BM_EINVAL),
        ("public key of another context", lambda: bm.bm_encrypt_query(ctx, pk2, one(16), 1, 1), bm.BM_EINVAL),
        ("add across contexts", lambda: bm.bm_op_add(ctx, q16, q2), bm.BM_EINVAL),
        ("decrypt with another context's key", lambda: bm.bm_decrypt_scores(ctx, sk2, r, 10), bm.BM_EINVAL),
        ("batch with a query of another context",
         lambda: bm.bm_match_batch(ctx, evk, [q16, q2], [g, g], schedule=1), bm.BM_EINVAL),
    ]
    for name, f, want in cases:
        got = status(f)
        assert got == want, "%s: status %d, expected %d" % (name, got, want)
    # the server keeps a rejected query with the caller
    srv = bm.bm_server_create(ctx, evk, 64 << 30, 1)
    gid = bm.bm_server_add_gallery(srv, g)
    assert status(lambda: bm.bm_server_submit(srv, gid, q8)) == bm.BM_EDIM
    assert status(lambda: bm.bm_server_submit(srv, gid, q2)) == bm.BM_EINVAL
    assert status(lambda: bm.bm_server_create(ctx, evk2, 64 << 30, 1)) == bm.BM_EINVAL
    bm.bm_server_free(srv)
    bm.bm_ct_free(q2)
    for f, h in ((bm.bm_sk_free, sk2), (bm.bm_pk_free, pk2), (bm.bm_evk_free, evk2)):
        f(h)
    bm.bm_ctx_free(ctx2)
    for h in (q16, q8, a, b, c2, c1):
        bm.bm_ct_free(h)
    bm.bm_result_free(r)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
        f(h)
    bm.bm_ctx_free(ctx)
    print("input checks ok", flush=True)


def server_from_threads():
    """bm_server_submit and bm_server_poll from several threads at once (the
    thread-safe pair): every ticket completes exactly once."""
    import threading
    p = bm.bm_params_preset(1)
    ctx = bm.bm_ctx_create(p, 0)
    sk, pk, evk = bm.bm_keygen(ctx, 1, sorted(set(bm.bm_rotations_for(16, 1)) | set(bm.bm_rotations_for(16, 4))))
    rng = np.random.default_rng(4)
    srv = bm.bm_server_create(ctx, evk, 64 << 30, 2 | bm.BM_LEVEL_MIN)
    gids = [bm.bm_server_add_gallery(srv, bm.bm_encrypt_gallery(ctx, pk, rng.standard_normal((n, 16)).astype(np.float32),
                                                                 k, 1, 10 * n))
            for n, k in ((300, 1), (700, 4))]
    n_threads, per = 4, 6
    queries = [[bm.bm_encrypt_query(ctx, pk, rng.standard_normal(16).astype(np.float32), 1, 100 * t + i)
                for i in range(per)] for t in range(n_threads)]   # the context itself is single-threaded
    done, errors = [0] * n_threads, []

    def client(t):
        try:
            tickets = [bm.bm_server_submit(srv, gids[(t + i) % 2], queries[t][i]) for i in range(per)]
            assert len(set(tickets)) == per
            pending = set(tickets)
            while pending:
                for tk in list(pending):
                    r = bm.bm_server_poll(srv, tk)
                    if r is not None:
                        bm.bm_result_free(r)
                        pending.discard(tk)
                        done[t] += 1
        except Exception as e:   # reported by the main thread
            errors.append(e)
    threads = [threading.Thread(target=client, args=(t,)) for t in range(n_threads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=300)
    assert not errors, errors
    assert done == [per] * n_threads, done
    assert bm.bm_server_stats(srv)["completed"] == n_threads * per
    # a served result belongs to the caller's context: it decrypts there
    tk = bm.bm_server_submit(srv, gids[0], bm.bm_encrypt_query(ctx, pk, rng.standard_normal(16).astype(np.float32),
                                                                 1, 999))
    bm.bm_server_drain(srv)
    r = bm.bm_server_poll(srv, tk)
    bm.bm_decrypt_scores(ctx, sk, r, 300)
    bm.bm_result_free(r)
    bm.bm_server_free(srv)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
        f(h)
    bm.bm_ctx_free(ctx)
    print("server from threads ok", flush=True)


def _is_prime(n):
    if n < 2 or n % 2 == 0:
        return n == 2
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1) or a % n == 0:
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _primes_below(bits, M, count):
    out, c = [], ((1 << bits) - 1) // M * M + 1
    while len(out) < count:
        if c < (1 << bits) and _is_prime(c):
            out.append(c)
        c -= M
    return out


def generic_rings():
    """Ring degrees other than the presets' (the generic integer transform):
    transforms, a match at every schedule, expansion and rotations."""
    for log_n in (10, 13):
        N = 1 << log_n
        p = bm.bm_params_preset(1)
        p.log_n = log_n
        for i, v in enumerate(_primes_below(50, 2 * N, 1) + _primes_below(40, 2 * N, 2)):
            p.q[i] = v
        p.p[0] = _primes_below(51, 2 * N, 1)[0]
        ctx = bm.bm_ctx_create(p, 0)
        rots = sorted(set(bm.bm_rotations_for(16, 1)) | set(bm.bm_rotations_for(16, 2)))
        sk, pk, evk = bm.bm_keygen(ctx, 1, rots)
        rng = np.random.default_rng(log_n)
        for k in (1, 2):
            X = rng.standard_normal((N // 16 + 7, 16)).astype(np.float32)
            q = bm.bm_encrypt_query(ctx, pk, X[0], 1, 1)
            g = bm.bm_encrypt_gallery(ctx, pk, X, k, 1, 10)
            for s in (1, 2, 1 | bm.BM_LEVEL_MIN):
                r = bm.bm_match(ctx, evk, q, g, None, schedule=s, out_limbs=0)
                bm.bm_decrypt_scores(ctx, sk, r, X.shape[0])
                bm.bm_result_free(r)
            bm.bm_ct_free(q)
            bm.bm_gallery_free(g)
        for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
            f(h)
        bm.bm_ctx_free(ctx)
        print("ring N=2^%d ok" % log_n, flush=True)


def key_import():
    """Keys exported in the coefficient domain and imported again; the host
    rejects malformed key words."""
    p = bm.bm_params_preset(1)
    ctx = bm.bm_ctx_create(p, 0)
    rots = bm.bm_rotations_for(16, 1)
    sk, pk, evk = bm.bm_keygen(ctx, 1, rots)
    gal = bm.bm_evk_galois(evk)
    assert len(gal) == len(set(rots)) and gal == sorted(gal)
    N, L1, npr = p.N, p.n_q, p.n_q + p.n_p
    dnum = -(-p.n_q // p.alpha)
    pkw = np.stack([bm.bm_pk_export(ctx, pk, c, L1, N) for c in (0, 1)])
    evw = np.stack([np.stack([np.stack([bm.bm_evk_export(ctx, evk, g, j, c, npr, N) for c in (0, 1)])
                              for j in range(dnum)]) for g in [0] + gal])
    pk2 = bm.bm_pk_import(ctx, np.zeros_like(pkw))
    evk2 = bm.bm_evk_import(ctx, gal, np.zeros_like(evw))
    assert bm.bm_evk_galois(evk2) == gal

    def status(f):
        try:
            f()
        except bm.BMError as e:
            return e.code
        return bm.BM_OK
    big = np.zeros_like(pkw)
    big[1, 2, 5] = p.q[2]                      # not a residue of its limb's prime
    cases = [
        ("public key of the wrong size", lambda: bm.bm_pk_import(ctx, pkw[:, :2]), bm.BM_EINVAL),
        ("public key word not reduced", lambda: bm.bm_pk_import(ctx, big), bm.BM_EINVAL),
        ("evaluation key of the wrong size", lambda: bm.bm_evk_import(ctx, gal, evw[:-1]), bm.BM_EINVAL),
        ("even Galois element", lambda: bm.bm_evk_import(ctx, [2] + gal[1:], evw), bm.BM_EINVAL),
        ("repeated Galois element", lambda: bm.bm_evk_import(ctx, [gal[0]] * len(gal), evw), bm.BM_EINVAL),
        ("Galois element out of range", lambda: bm.bm_evk_import(ctx, [2 * N + 1] + gal[1:], evw), bm.BM_EINVAL),
    ]
    for name, f, want in cases:
        got = status(f)
        assert got == want, "%s: status %d, expected %d" % (name, got, want)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk), (bm.bm_pk_free, pk2),
                 (bm.bm_evk_free, evk2)):
        f(h)
    bm.bm_ctx_free(ctx)
    print("key import ok", flush=True)


def result_outlives_server():
    """A served result freed after its server: its memory came from a server
    lane, which the result keeps alive."""
    p = bm.bm_params_preset(1)
    ctx = bm.bm_ctx_create(p, 0)
    sk, pk, evk = bm.bm_keygen(ctx, 1, bm.bm_rotations_for(16, 1))
    X = np.ones((40, 16), dtype=np.float32)
    srv = bm.bm_server_create(ctx, evk, 64 << 30, 2)
    gid = bm.bm_server_add_gallery(srv, bm.bm_encrypt_gallery(ctx, pk, X, 1, 1, 10))
    tk = bm.bm_server_submit(srv, gid, bm.bm_encrypt_query(ctx, pk, X[0], 1, 1))
    bm.bm_server_drain(srv)
    r = bm.bm_server_poll(srv, tk)
    bm.bm_server_free(srv)
    bm.bm_decrypt_scores(ctx, sk, r, 40)
    bm.bm_result_free(r)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
        f(h)
    bm.bm_ctx_free(ctx)
    print("result outlives server ok", flush=True)


def noalloc_flow():
    """The no-allocation match: size query, host-side refusals, a match that
    needs more scratch than the array holds (refused before any launch), and
    the launch checks of matches that fit, on host buffers standing in for
    device ones."""
    for preset, shapes in ((1, [(16, 1, 0x001), (16, 4, 0x002), (16, 4, 0x402)]),
                           (2, [(128, 4, 0x102), (16, 1, 0x101), (128, 16, 0x002)])):
        p = bm.bm_params_preset(preset)
        ctx = bm.bm_ctx_create(p, 0)
        rots = set()
        for d, k, _ in shapes:
            rots.update(bm.bm_rotations_for(d, k))
            rots.update(bm.bm_rotations_hoisted(d, k))
        sk, pk, evk = bm.bm_keygen(ctx, 1, sorted(rots))
        rng = np.random.default_rng(1)
        q = np.zeros((2, p.n_q, p.N), dtype=np.uint64)
        for d, k, s in shapes:
            X = rng.standard_normal((700, d)).astype(np.float32)
            g = bm.bm_encrypt_gallery(ctx, pk, X, k, 1, 10)
            if k == 1:
                m = None
            elif s & bm.BM_LEVEL_MIN:           # masks at the scale of the query cut to 4 limbs
                m = bm.bm_masks_import(ctx, d, k, np.zeros((k, p.N), dtype=np.int64), float(p.chain()[3]))
            else:
                m = bm.bm_masks_create(ctx, d, k)
            need, _ = bm.bm_match_noalloc(ctx, evk, q.ctypes.data, p.n_q, p.scale, g, m, s, 0)
            out = np.zeros(need, dtype=np.uint64)
            try:
                bm.bm_match_noalloc(ctx, evk, q.ctypes.data, p.n_q, p.scale, g, m, s, 0, out.ctypes.data, need)
                assert not (preset == 2 and k == 16), "a match above the scratch size was accepted"
            except bm.BMError as e:
                assert preset == 2 and k == 16 and e.code == bm.BM_ENOMEM, e
            for bad, code in (((need - 1,), bm.BM_EINVAL),):
                try:
                    bm.bm_match_noalloc(ctx, evk, q.ctypes.data, p.n_q, p.scale, g, m, s, 0, out.ctypes.data, *bad)
                    raise AssertionError("wrong output size accepted")
                except bm.BMError as e:
                    assert e.code == code
            if k > 1:
                try:
                    bm.bm_match_noalloc(ctx, evk, q.ctypes.data, p.n_q, p.scale, g, None, s, 0, out.ctypes.data, need)
                    raise AssertionError("k > 1 without masks accepted")
                except bm.BMError as e:
                    assert e.code == bm.BM_EINVAL
                bm.bm_masks_free(m)
            bm.bm_gallery_free(g)
        for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
            f(h)
        bm.bm_ctx_free(ctx)
    print("no-allocation match ok", flush=True)


def tuning_flow():
    """Every kernel variant and row-pass tiling of the tuning knobs at every
    digit count the hoisted sums meet, the batch autotuner, and a batch of
    mixed shapes with graphs on and off."""
    for preset, shapes in ((1, [(16, 1), (16, 4), (8, 8)]), (2, [(16, 1), (128, 4), (64, 2)])):
        p = bm.bm_params_preset(preset)
        ctx = bm.bm_ctx_create(p, 0)
        rots = set()
        for d, k in shapes:
            rots.update(bm.bm_rotations_for(d, k))
            rots.update(bm.bm_rotations_hoisted(d, k))
        sk, pk, evk = bm.bm_keygen(ctx, 1, sorted(rots))
        rng = np.random.default_rng(2)
        qs, gs = [], []
        for d, k in shapes:
            for n in (300, 1300):
                g = bm.bm_encrypt_gallery(ctx, pk, rng.standard_normal((n, d)).astype(np.float32), k, 1, n)
                for j in range(2):
                    qs.append(bm.bm_encrypt_query(ctx, pk, rng.standard_normal(d).astype(np.float32), 1, 10 * n + j))
                    gs.append(g)
        for var in range(5):
            for views, order, occ, src in ((0, 0, 0, 0), (4, 1, 4, 1), (8, 2, 3, 0), (16, 3, 0, 1)):
                bm.bm_ctx_set_tuning(ctx, group_chunk=3, kip_variant=var, ntt_row_views=views, kip_order=order,
                                     fused_occupancy=occ, column_sources=src)
                # natural level (hoisted sums at 2 to 4 digits) and minimum level (1 digit)
                for s in (0x402, 0x502, 0x401):
                    for r in bm.bm_match_batch(ctx, evk, qs, gs, schedule=s):
                        bm.bm_result_free(r)
        for graphs in (0, 1):
            bm.bm_ctx_set_graphs(ctx, graphs)
            for r in bm.bm_match_batch(ctx, evk, qs, gs, schedule=0x102, out_limbs=1):
                bm.bm_result_free(r)
        bm.bm_ctx_set_graphs(ctx, False)
        sched, tun, ms = bm.bm_autotune_batch(ctx, evk, qs, gs, [0x102, 0x502, 0x002], out_limbs=0)
        assert sched in (0x102, 0x502, 0x002), sched
        assert bm.bm_ctx_get_tuning(ctx) == tun
        try:
            bm.bm_autotune_batch(ctx, evk, qs, gs, [0x7777])
            raise AssertionError("unknown schedule flags accepted")
        except bm.BMError as e:
            assert e.code == bm.BM_EINVAL
        for q in qs:
            bm.bm_ct_free(q)
        for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
            f(h)
        bm.bm_ctx_free(ctx)
    print("tuning ok", flush=True)


if __name__ == "__main__":
    tuning_flow()
    noalloc_flow()
    result_outlives_server()
    key_import()
    generic_rings()
    server_from_threads()
    input_checks()
    allocator_hook_flow()
    flow(1, [(16, 1), (16, 2), (16, 4), (8, 8)], 300)
    flow(2, [(128, 1), (128, 4), (128, 16), (16, 1)], 5000)
    # conjugate-invariant ring (N real slots)
    flow(3, [(16, 1), (16, 4), (8, 8)], 600)
    flow(4, [(128, 4), (128, 16)], 9000)
    print("dry run ok")
