"""GPU: a context whose device memory comes from torch's caching allocator
(bm_ctx_set_allocator) computes the same words as one on the library's own
allocation -- eager, replayed as a HIP graph and through a server lane -- and
gives every block back when it is freed."""
import numpy as np
import pytest

from gpu_common import SEED, all_rotations, assert_words_equal, log
from workloads import normalize

pytestmark = pytest.mark.gpu

D, K, N_TEMPLATES = 16, 4, 300


def words_of(bm, ctx, res, N):
    G, _, _ = bm.bm_result_info(res)
    return [bm.bm_result_export(ctx, res, g, N)[0] for g in range(G)]


def run(bm, torch, hooked):
    p = bm.bm_params_preset(1)
    ctx = bm.bm_ctx_create(p, 0)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    calls = dict(alloc=0, free=0)
    if hooked:
        t_alloc, t_free = bm.torch_allocator(0)

        def alloc(n):
            calls["alloc"] += 1
            return t_alloc(n)

        def free(ptr):
            calls["free"] += 1
            t_free(ptr)
        bm.bm_ctx_set_allocator(ctx, alloc, free)
    sk, pk, evk = bm.bm_keygen(ctx, SEED, all_rotations(1, [(D, K)]))
    if hooked:
        # every block the pool holds came from torch
        assert calls["alloc"] > 0
        assert torch.cuda.memory_allocated(0) - base >= bm.bm_ctx_pool_bytes(ctx)
    rng = np.random.default_rng(5)
    X = normalize(rng.standard_normal((N_TEMPLATES, D)))
    g = bm.bm_encrypt_gallery(ctx, pk, X, K, SEED, 100)
    q = bm.bm_encrypt_query(ctx, pk, X[17], SEED, 1)
    out = {}
    for graphs in (False, True):
        bm.bm_ctx_set_graphs(ctx, graphs)
        for rep in range(2):
            r = bm.bm_match(ctx, evk, q, g, None, schedule=2)
            out[(graphs, rep)] = words_of(bm, ctx, r, p.N)
            if rep == 0 and not graphs:
                s = bm.bm_decrypt_scores(ctx, sk, r, N_TEMPLATES)
                assert int(np.argmax(s)) == 17
            bm.bm_result_free(r)
    bm.bm_ctx_set_graphs(ctx, False)
    # a server lane (its own pool, allocating from a worker thread)
    srv = bm.bm_server_create(ctx, evk, 64 << 30, 2)
    gid = bm.bm_server_add_gallery(srv, g)          # the server owns the gallery now
    t = bm.bm_server_submit(srv, gid, bm.bm_encrypt_query(ctx, pk, X[17], SEED, 1))
    bm.bm_server_drain(srv)
    r = bm.bm_server_poll(srv, t)
    out["server"] = words_of(bm, ctx, r, p.N)
    bm.bm_result_free(r)
    bm.bm_server_free(srv)
    bm.bm_ct_free(q)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
        f(h)
    bm.bm_ctx_free(ctx)
    torch.cuda.synchronize()
    if hooked:
        assert calls["free"] == calls["alloc"], calls
        assert torch.cuda.memory_allocated(0) == base
    return out


def test_torch_allocator_same_words_and_all_returned():
    import torch
    import paper_2408_06167_amd as bm
    log("allocator hook: own allocation")
    want = run(bm, torch, False)
    log("allocator hook: torch caching allocator")
    got = run(bm, torch, True)
    assert set(got) == set(want)
    for key in want:
        assert len(got[key]) == len(want[key])
        for gi, (a, b) in enumerate(zip(got[key], want[key])):
            assert_words_equal(a, b, "%s group %d" % (key, gi))
    for key in want:   # eager, replayed and served matches agree with each other too
        for gi, (a, b) in enumerate(zip(want[key], want[(False, 0)])):
            assert_words_equal(a, b, "%s vs eager, group %d" % (key, gi))
