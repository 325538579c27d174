"""GPU: the no-allocation match (bm_match_noalloc) against bm_match.

The entry point runs the match of bm_match on caller-owned device buffers
with its scratch carved out of the library's per-device scratch array.  Its
words must equal bm_match's on the same inputs (exact integer arithmetic: the
bar is bit-identity), on two calls in a row of which the second has a smaller
input, and a call whose scratch need exceeds the array must fail before it
enqueues anything."""
import numpy as np
import pytest

from gpu_common import SEED, lib_ctx, assert_words_equal, log
from workloads import normalize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bm():
    import paper_2408_06167_amd as bm
    return bm


def device_query(bm, ctx, ct, p, stream):
    """Evaluation-domain words of a query ciphertext in a torch device tensor."""
    import torch
    words, scale = bm.bm_ct_export(ctx, ct, p.N)
    comps, limbs, _ = words.shape
    dev = torch.from_numpy(words.view(np.int64).copy()).cuda()
    bm.bm_ntt(ctx, dev.data_ptr(), comps, list(range(limbs)), False, stream)
    return dev, limbs, scale


def noalloc_words(bm, ctx, evk, qdev, q_limbs, q_scale, gal, masks, schedule, out_limbs, p, stream):
    """Run the no-allocation match; its output converted to coefficient words
    [G][2][ol][N] on the host, and the result scale."""
    import torch
    need, _ = bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), q_limbs, q_scale, gal, masks, schedule, out_limbs)
    G = bm.bm_gallery_info(gal)[0]
    assert need % (G * 2 * p.N) == 0
    ol = need // (G * 2 * p.N)
    out = torch.full((need,), -1, dtype=torch.int64, device="cuda")
    _, scale = bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), q_limbs, q_scale, gal, masks, schedule, out_limbs,
                                   out.data_ptr(), need, stream)
    bm.bm_ntt(ctx, out.data_ptr(), G * 2, list(range(ol)), True, stream)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64).reshape(G, 2, ol, p.N), scale


def plain_words(bm, ctx, evk, q, gal, masks, schedule, out_limbs, p):
    r = bm.bm_match(ctx, evk, q, gal, masks, schedule=schedule, out_limbs=out_limbs)
    G, limbs, scale = bm.bm_result_info(r)
    w = np.stack([bm.bm_result_export(ctx, r, g, p.N)[0] for g in range(G)])
    bm.bm_result_free(r)
    return w, scale


def level_masks(bm, ctx, p, d, k, limbs):
    """The library's Alg. 1 masks re-made at scale q_{limbs-1}: a query cut to
    `limbs` limbs (minimum-level schedule) multiplies masks at that scale."""
    from oracle import ckks, blindmatch as obm
    P = ckks.Params.preset(2 if p.log_n == 16 else 1)
    coeffs, scale = obm.mask_coeffs(P, d, k, limbs)
    return bm.bm_masks_import(ctx, d, k, np.stack(coeffs), scale)


# (preset, d, k, schedule, out_limbs, templates of the first call, of the second)
CASES = [(1, 16, 1, 0x001, 0, 300, 100), (1, 16, 4, 0x002, 0, 1300, 500), (1, 16, 4, 0x402, 0, 1300, 200),
         (2, 128, 4, 0x502, 2, 6144, 1500), (2, 16, 1, 0x101, 2, 5000, 900)]


@pytest.mark.parametrize("preset,d,k,schedule,out_limbs,n1,n2", CASES)
def test_noalloc_match_equals_bm_match(bm, preset, d, k, schedule, out_limbs, n1, n2):
    import torch
    ctx = lib_ctx(preset)
    p = bm.bm_params_preset(preset)
    rots = set(bm.bm_rotations_for(d, k))
    if schedule & bm.BM_HOIST:
        rots.update(bm.bm_rotations_hoisted(d, k))
    sk, pk, evk = bm.bm_keygen(ctx, SEED + 7, sorted(rots))
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(n1 + d + k)
    lmin = bool(schedule & bm.BM_LEVEL_MIN)
    masks = None
    if k > 1:
        ql = (3 + 1) if lmin else p.n_q
        masks = level_masks(bm, ctx, p, d, k, ql) if lmin else bm.bm_masks_create(ctx, d, k)
    for call, n in enumerate((n1, n2)):                 # two calls, the second with a smaller gallery
        X = normalize(rng.standard_normal((n, d)))
        qv = normalize(X[n // 2] + 0.05 * rng.standard_normal(d))
        q = bm.bm_encrypt_query(ctx, pk, qv, SEED, 60 + call)
        gal = bm.bm_encrypt_gallery(ctx, pk, X, k, SEED, 9000 + 1000 * call)
        log("noalloc preset %d d=%d k=%d schedule %#x call %d (%d templates)" % (preset, d, k, schedule, call, n))
        qdev, ql_, qs = device_query(bm, ctx, q, p, stream)
        got, gscale = noalloc_words(bm, ctx, evk, qdev, ql_, qs, gal, masks, schedule, out_limbs, p, stream)
        want, wscale = plain_words(bm, ctx, evk, q, gal, masks, schedule, out_limbs, p)
        assert gscale == wscale
        assert_words_equal(got, want, "call %d" % call)
        bm.bm_ct_free(q)
        bm.bm_gallery_free(gal)
    if masks:
        bm.bm_masks_free(masks)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
        f(h)


def test_noalloc_rejections(bm):
    """Sizes, missing masks, compression, and a match whose scratch need
    exceeds the array: an error, and the output buffer left untouched."""
    import torch
    ctx = lib_ctx(2)
    p = bm.bm_params_preset(2)
    d, k = 128, 16
    sk, pk, evk = bm.bm_keygen(ctx, SEED + 8, sorted(set(bm.bm_rotations_for(d, k))))
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(3)
    X = normalize(rng.standard_normal((2000, d)))
    q = bm.bm_encrypt_query(ctx, pk, X[0], SEED, 1)
    gal = bm.bm_encrypt_gallery(ctx, pk, X, k, SEED, 100)
    masks = bm.bm_masks_create(ctx, d, k)
    qdev, ql, qs = device_query(bm, ctx, q, p, stream)
    need, _ = bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), ql, qs, gal, masks, 2, 2)
    out = torch.full((need,), 7, dtype=torch.int64, device="cuda")

    def status(f):
        try:
            f()
        except bm.BMError as e:
            return e.code
        return bm.BM_OK
    assert status(lambda: bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), ql, qs, gal, masks, 2, 2,
                                              out.data_ptr(), need - 1)) == bm.BM_EINVAL
    assert status(lambda: bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), ql, qs, gal, None, 2, 2,
                                              out.data_ptr(), need)) == bm.BM_EINVAL
    assert status(lambda: bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), ql, qs, gal, masks, 2 | bm.BM_COMPRESS, 2,
                                              out.data_ptr(), need)) == bm.BM_EINVAL
    # k = 16 at the natural level expands 16 parts at 8 limbs: more than the scratch holds
    assert status(lambda: bm.bm_match_noalloc(ctx, evk, qdev.data_ptr(), ql, qs, gal, masks, 2, 2,
                                              out.data_ptr(), need, stream)) == bm.BM_ENOMEM
    torch.cuda.synchronize()
    assert bool((out == 7).all()), "a refused call wrote its output"
    bm.bm_masks_free(masks)
    bm.bm_ct_free(q)
    bm.bm_gallery_free(gal)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk)):
        f(h)
